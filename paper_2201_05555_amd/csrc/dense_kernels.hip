// Single-workgroup FP64 kernels on the small dense matrices of a reduced
// step (n x n, 2n x 2n, n x p): S(Z)^+ (Sec. 3.2), the Woodbury system of the
// Cayley retraction and the inverses of the tangent velocity (Sec. 5), the
// Cholesky factor of the re-orthonormalisation, and the per-column
// fixed-point control.  Everything is in the complex representation:
// a real 2n x 2n matrix that commutes with J_2n is the n x n complex matrix
// A + iB of its blocks [[A, -B], [B, A]].
//
// Matrices are column-major.  `flags` words: [0] error bits (1 = singular LU,
// 2 = Cholesky breakdown), [1] 1 if the Jacobi eigen path was taken.
#include "common.h"
#include "kernels.h"

#define DTPB 256
// complex entries of an n x p coefficient block staged in LDS by the dense
// kernels (64 KB); larger blocks are read in place
#define DENSE_Z_LDS 4096

// ---------------------------------------------------------------------------
// block-cooperative helpers (all threads of the block call them)
// ---------------------------------------------------------------------------

// C (m x n) = op(A) op(B), op = identity (0) or conjugate transpose (1).
// A is stored m x k (opA = 0) or k x m (opA = 1); B is k x n or n x k.
__device__ void bk_matmul(cplx* C, const cplx* A, int opA, const cplx* B, int opB, int m, int k,
                          int n) {
  for (int t = threadIdx.x; t < m * n; t += blockDim.x) {
    int i = t % m, j = t / m;
    cplx s = mk(0.0, 0.0);
    for (int q = 0; q < k; ++q) {
      cplx a = opA ? cconj(A[i * k + q]) : A[q * m + i];
      cplx b = opB ? cconj(B[q * n + j]) : B[j * k + q];
      cfma(s, a, b);
    }
    C[j * m + i] = s;
  }
  __syncthreads();
}

// Entry (i, j) of A B for column-major n x n A, B, summed in the order of
// bk_matmul (so a product formed entry by entry has the same bits).
__device__ inline cplx mm_entry(const cplx* A, const cplx* B, int i, int j, int n) {
  cplx s = mk(0.0, 0.0);
  for (int q = 0; q < n; ++q) cfma(s, A[q * n + i], B[j * n + q]);
  return s;
}

// Solve A X = B in place (A m x m destroyed, B m x nrhs overwritten by X)
// by Gaussian elimination with partial pivoting.  Returns 0 on success.
__device__ int bk_lu_solve(cplx* A, int m, cplx* B, int nrhs, int* piv_s) {
  __shared__ int fail;
  if (threadIdx.x == 0) fail = 0;
  __syncthreads();
  for (int c = 0; c < m; ++c) {
    if (threadIdx.x == 0) {
      int best = c;
      double bv = cabs2(A[c * m + c]);
      // four independent LDS loads per round, compared in row order
      int r = c + 1;
      for (; r + 3 < m; r += 4) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = cabs2(A[c * m + r + u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (v[u] > bv) {
            bv = v[u];
            best = r + u;
          }
      }
      for (; r < m; ++r) {
        double v = cabs2(A[c * m + r]);
        if (v > bv) {
          bv = v;
          best = r;
        }
      }
      if (!(bv > 0.0)) fail = 1;
      *piv_s = best;
    }
    __syncthreads();
    if (fail) return 1;
    const int pr = *piv_s;
    if (pr != c) {
      for (int j = threadIdx.x; j < m + nrhs; j += blockDim.x) {
        cplx* col = (j < m) ? A + j * m : B + (j - m) * m;
        cplx t = col[c];
        col[c] = col[pr];
        col[pr] = t;
      }
    }
    __syncthreads();
    const cplx piv = A[c * m + c];
    const double pn = cabs2(piv);
    const cplx pinv = mk(piv.re / pn, -piv.im / pn);
    // eliminate below the pivot: rows r > c, columns j > c of A and all of B
    const int rows = m - c - 1;
    const int cols = (m - c - 1) + nrhs;
    for (int t = threadIdx.x; t < rows * cols; t += blockDim.x) {
      int r = c + 1 + t % rows;
      int jj = t / rows;
      cplx f = cmul(A[c * m + r], pinv);
      cplx* col = (jj < m - c - 1) ? A + (c + 1 + jj) * m : B + (jj - (m - c - 1)) * m;
      col[r] = csub(col[r], cmul(f, col[c]));
    }
    __syncthreads();
  }
  // back substitution, one barrier per column: x_c = B[c] / A[c][c] is
  // recomputed by every thread that eliminates with it (row c itself is not
  // written until the end), then all rows are scaled in one pass
  for (int c = m - 1; c >= 1; --c) {
    const cplx piv = A[c * m + c];
    const double pn = cabs2(piv);
    const cplx pinv = mk(piv.re / pn, -piv.im / pn);
    for (int t = threadIdx.x; t < c * nrhs; t += blockDim.x) {
      int r = t % c, j = t / c;
      const cplx xc = cmul(B[j * m + c], pinv);
      B[j * m + r] = csub(B[j * m + r], cmul(A[c * m + r], xc));
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < m * nrhs; t += blockDim.x) {
    const int c = t % m;
    const cplx piv = A[c * m + c];
    const double pn = cabs2(piv);
    B[t] = cmul(B[t], mk(piv.re / pn, -piv.im / pn));
  }
  __syncthreads();
  return 0;
}

// Upper Cholesky G = R^* R (G n x n Hermitian, R overwrites a separate
// buffer, lower part zero).  Returns 0 on success, 1 if a pivot is not
// positive.  `shift` is subtracted from the diagonal first.
__device__ int bk_chol(const cplx* G, cplx* R, int n, double shift) {
  __shared__ int fail;
  if (threadIdx.x == 0) fail = 0;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) R[t] = mk(0.0, 0.0);
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double d = G[j * n + j].re - shift;
#pragma unroll 4
      for (int k = 0; k < j; ++k) d -= cabs2(R[j * n + k]);
      if (!(d > 0.0)) {
        fail = 1;
        d = 1.0;
      }
      R[j * n + j] = mk(sqrt(d), 0.0);
    }
    __syncthreads();
    if (fail) return 1;
    const double rjj = R[j * n + j].re;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) {
      cplx s = G[i * n + j];  // G[j][i]
      for (int k = 0; k < j; ++k) s = csub(s, cmulc(R[j * n + k], R[i * n + k]));
      R[i * n + j] = cscale(s, 1.0 / rjj);
    }
    __syncthreads();
  }
  return 0;
}

// Inverse of an upper triangular R (n x n) into Ri (upper).
__device__ void bk_triu_inv(const cplx* R, cplx* Ri, int n) {
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) Ri[t] = mk(0.0, 0.0);
  __syncthreads();
  // column j of Ri solves R x = e_j, x upper; threads over columns
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    for (int i = j; i >= 0; --i) {
      cplx s = (i == j) ? mk(1.0, 0.0) : mk(0.0, 0.0);
      for (int k = i + 1; k <= j; ++k) s = csub(s, cmul(R[k * n + i], Ri[j * n + k]));
      const cplx d = R[i * n + i];
      const double dn = cabs2(d);
      Ri[j * n + i] = cmul(s, mk(d.re / dn, -d.im / dn));
    }
  }
  __syncthreads();
}

// Parallel cyclic Jacobi for a Hermitian m x m matrix A (overwritten; its
// diagonal ends as the eigenvalues), V receives the eigenvectors.  Pairs of
// one round are disjoint (round-robin ordering), so their rotations are
// applied together: first A <- A G, then A <- G^* A, then V <- V G.
// Eigenvalues are returned in lam sorted in decreasing order, with the
// columns of V permuted to match.
__device__ void bk_jacobi(cplx* A, cplx* V, double* lam, int m, cplx* rot /*3*m/2+3*/,
                          int* pr /*m+2*/) {
  const int mm = m + (m & 1);
  const int half = mm / 2;
  for (int t = threadIdx.x; t < m * m; t += blockDim.x)
    V[t] = (t % m == t / m) ? mk(1.0, 0.0) : mk(0.0, 0.0);
  __shared__ double red[DTPB / 64];
  __shared__ int nrot;
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    // threshold Jacobi: an off-diagonal entry is rotated away only when it is
    // above 1e-15 sqrt(|a_pp a_qq|) and above 1e-18 of the largest diagonal
    // entry; the sweep loop ends when a sweep applies no rotation
    double dmax = 0.0;
    for (int t = threadIdx.x; t < m; t += blockDim.x) dmax = fmax(dmax, fabs(A[t * m + t].re));
    for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dmax;
    if (threadIdx.x == 0) nrot = 0;
    __syncthreads();
    dmax = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) dmax = fmax(dmax, red[w]);
    const double floor_abs = 1e-18 * dmax;
    __syncthreads();
    for (int round = 0; round < mm - 1; ++round) {
      for (int k = threadIdx.x; k < half; k += blockDim.x) {
        int a, b;
        if (k == 0) {
          a = mm - 1;
          b = round;
        } else {
          a = (round + k) % (mm - 1);
          b = (round - k + (mm - 1)) % (mm - 1);
        }
        int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        cplx ph = mk(1.0, 0.0);  // e^{-i phi}
        if (q < m) {
          const cplx bpq = A[q * m + p];
          const double ab = sqrt(cabs2(bpq));
          const double app = A[p * m + p].re, aqq = A[q * m + q].re;
          if (ab > 1e-300 && ab > floor_abs && ab > 1e-15 * sqrt(fabs(app * aqq))) {
            atomicAdd(&nrot, 1);
            ph = mk(bpq.re / ab, -bpq.im / ab);
            const double zeta = (aqq - app) / (2.0 * ab);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pr[2 * k] = p;
        pr[2 * k + 1] = q;
        rot[3 * k] = mk(c, s);
        rot[3 * k + 1] = ph;
      }
      __syncthreads();
      // A <- A G  (columns p, q)
      for (int t = threadIdx.x; t < m * half; t += blockDim.x) {
        int r = t % m, k = t / m;
        int p = pr[2 * k], q = pr[2 * k + 1];
        if (q >= m) continue;
        double c = rot[3 * k].re, s = rot[3 * k].im;
        if (s == 0.0) continue;
        cplx ph = rot[3 * k + 1];
        cplx x = A[p * m + r], y = A[q * m + r];
        cplx yph = cmul(y, ph);
        A[p * m + r] = csub(cscale(x, c), cscale(yph, s));
        A[q * m + r] = cadd(cscale(x, s), cscale(yph, c));
      }
      __syncthreads();
      // A <- G^* A  (rows p, q)
      for (int t = threadIdx.x; t < m * half; t += blockDim.x) {
        int col = t % m, k = t / m;
        int p = pr[2 * k], q = pr[2 * k + 1];
        if (q >= m) continue;
        double c = rot[3 * k].re, s = rot[3 * k].im;
        if (s == 0.0) continue;
        cplx phc = cconj(rot[3 * k + 1]);  // e^{+i phi}
        cplx x = A[col * m + p], y = A[col * m + q];
        cplx yph = cmul(y, phc);
        A[col * m + p] = csub(cscale(x, c), cscale(yph, s));
        A[col * m + q] = cadd(cscale(x, s), cscale(yph, c));
      }
      __syncthreads();
      // V <- V G
      for (int t = threadIdx.x; t < m * half; t += blockDim.x) {
        int r = t % m, k = t / m;
        int p = pr[2 * k], q = pr[2 * k + 1];
        if (q >= m) continue;
        double c = rot[3 * k].re, s = rot[3 * k].im;
        if (s == 0.0) continue;
        cplx ph = rot[3 * k + 1];
        cplx x = V[p * m + r], y = V[q * m + r];
        cplx yph = cmul(y, ph);
        V[p * m + r] = csub(cscale(x, c), cscale(yph, s));
        V[q * m + r] = cadd(cscale(x, s), cscale(yph, c));
      }
      // the rotated diagonal entries are real in exact arithmetic
      for (int k = threadIdx.x; k < half; k += blockDim.x) {
        int p = pr[2 * k], q = pr[2 * k + 1];
        if (q < m) {
          A[p * m + p].im = 0.0;
          A[q * m + q].im = 0.0;
        }
      }
      __syncthreads();
    }
    if (nrot == 0) break;
    __syncthreads();
  }
  // sort eigenpairs by decreasing eigenvalue (selection by thread 0 of the
  // permutation, then parallel column moves through the rot scratch)
  if (threadIdx.x == 0) {
    for (int i = 0; i < m; ++i) {
      lam[i] = A[i * m + i].re;
      pr[i] = i;
    }
    for (int i = 0; i < m; ++i) {
      int b = i;
      for (int j = i + 1; j < m; ++j)
        if (lam[j] > lam[b]) b = j;
      double tl = lam[i];
      lam[i] = lam[b];
      lam[b] = tl;
      int tp = pr[i];
      pr[i] = pr[b];
      pr[b] = tp;
    }
  }
  __syncthreads();
  // permute V columns: out column i = old column pr[i]; use A as scratch
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) A[t] = V[t];
  __syncthreads();
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
    int r = t % m, i = t / m;
    V[i * m + r] = A[pr[i] * m + r];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// S(Z)^+ and Q = Z~^* S~^+ (p x n), with S~ = Z~ Z~^* (the complex form of
// S(Z) = Z Z^T + J^T Z Z^T J).  The Moore-Penrose inverse drops eigenvalues
// below rtol * lambda_max.  When S~ - rtol trace(S~) I admits a Cholesky
// factor, every eigenvalue exceeds rtol * lambda_max (lambda_max <= trace),
// nothing would be dropped and S~^+ = S~^{-1} is formed from the Cholesky
// factor; otherwise the Jacobi eigendecomposition is used.
// sigma2 receives the eigenvalues (decreasing) when the eigen path runs, else
// is left untouched.  Requires n <= 32.  Z is copied to LDS first (one
// coalesced pass), so that no loop waits on global loads.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(DTPB) dense_spinv_kernel(const cplx* __restrict__ Z, int n, int p,
                                                           double rtol, cplx* __restrict__ Q,
                                                           double* __restrict__ sigma2,
                                                           int* __restrict__ flags) {
  extern __shared__ cplx sm[];
  // Z (n x p) is staged in LDS when it fits (zlds), else read in place
  const bool zlds = n * p <= DENSE_Z_LDS;
  const cplx* Zs = zlds ? sm : Z;
  cplx* S = zlds ? sm + n * p : sm;   // n x n
  cplx* R = S + n * n;
  cplx* Ri = R + n * n;
  __shared__ cplx rot[3 * 17 + 3];
  __shared__ int pr[40];
  __shared__ double lam[32];
  __shared__ double trs;
  if (zlds) {
    for (int t = threadIdx.x; t < n * p; t += blockDim.x) sm[t] = Z[t];
    __syncthreads();
  }
  // S~ = Z~ Z~^*
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int a = t % n, b = t / n;
    cplx s = mk(0.0, 0.0);
    for (int i = 0; i < p; ++i) cfma(s, Zs[i * n + a], cconj(Zs[i * n + b]));
    S[t] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int a = 0; a < n; ++a) tr += S[a * n + a].re;
    trs = tr;
  }
  __syncthreads();
  int bad = bk_chol(S, R, n, rtol * trs);
  if (!bad) bad = bk_chol(S, R, n, 0.0);
  if (!bad) {
    // S^{-1} = R^{-1} R^{-*}
    bk_triu_inv(R, Ri, n);
    bk_matmul(R, Ri, 0, Ri, 1, n, n, n);  // R <- S^{-1}
    if (threadIdx.x == 0 && flags) flags[1] = 0;
  } else {
    // eigen path: S = V diag(lam) V^*
    bk_jacobi(S, Ri, lam, n, rot, pr);
    const double lmax = lam[0];
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
      int a = t % n, b = t / n;
      cplx s = mk(0.0, 0.0);
      for (int k = 0; k < n; ++k) {
        if (lam[k] > rtol * lmax) cfma(s, cscale(Ri[k * n + a], 1.0 / lam[k]), cconj(Ri[k * n + b]));
      }
      R[t] = s;
    }
    if (sigma2)
      for (int k = threadIdx.x; k < n; k += blockDim.x) sigma2[k] = lam[k];
    if (threadIdx.x == 0 && flags) flags[1] = 1;
    __syncthreads();
  }
  // Q[i, b] = sum_a conj(Z[a, i]) S^+[a, b]
  for (int t = threadIdx.x; t < p * n; t += blockDim.x) {
    int i = t % p, b = t / p;
    cplx s = mk(0.0, 0.0);
    for (int a = 0; a < n; ++a) cfma(s, cconj(Zs[i * n + a]), R[b * n + a]);
    Q[(size_t)b * p + i] = s;
  }
}

// After the full-gradient projection g~ = U~^* G~ (n x p): k1 = -i g~ and the
// row-combination matrices of xi = (dt/2) X~ with X~ = -i (P~ - U~ T),
// T = g~ Q (n x n):  xi = P~ (-i dt/2 I) + U~ (i dt/2 T).
// g and Q are copied to LDS first (one coalesced pass).
__global__ void __launch_bounds__(DTPB) dense_xfinish_kernel(const cplx* __restrict__ g,
                                                             const cplx* __restrict__ Q, int n,
                                                             int p, double dt, cplx* __restrict__ k1,
                                                             cplx* __restrict__ MP,
                                                             cplx* __restrict__ MU) {
  extern __shared__ cplx sm[];
  // g (n x p) and Q (p x n) staged in LDS when they fit, else read in place
  const bool lds = n * p <= DENSE_Z_LDS;
  const cplx* gs = lds ? sm : g;
  const cplx* Qs = lds ? sm + n * p : Q;
  for (int t = threadIdx.x; t < n * p; t += blockDim.x) {
    const cplx gv = g[t];
    if (lds) {
      sm[t] = gv;
      sm[n * p + t] = Q[t];
    }
    if (k1) k1[t] = mk(gv.im, -gv.re);
  }
  __syncthreads();
  const double h = 0.5 * dt;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int a = t % n, b = t / n;
    cplx s = mk(0.0, 0.0);
    for (int i = 0; i < p; ++i) cfma(s, gs[i * n + a], Qs[b * p + i]);
    MU[t] = mk(-h * s.im, h * s.re);  // i h T
    MP[t] = (a == b) ? mk(0.0, -h) : mk(0.0, 0.0);
  }
}

// Cayley retraction R_{U0}(xi) in complex form by Sherman-Morrison-Woodbury.
// Input: Gram = [U0, xi]^* [U0, xi] (2n x 2n).  With A = U0^* xi,
// W = xi - U0 A / 2, Lc = [W, -U0], Rc = [U0, W]:
//   K = (I - Rc^* Lc / 2)^{-1},  [Y1; Y2] = K Rc^* U0,
//   R_{U0}(xi) = U0 + W Y1 - U0 Y2 = U0 (I - Y2 - A Y1 / 2) + xi Y1.
// Output MU, MX (n x n) for the row combination, and A.
// chol: also one Cholesky-QR pass of R_{U0}(xi) without a pass over its rows.
// Its Gram is G1 = [MU; MX]^* Gram [MU; MX] = R^* R; MU, MX are returned
// multiplied by R^{-1} and Z (n x p, optional) is replaced by R Z.
__global__ void __launch_bounds__(DTPB) dense_cayley_kernel(const cplx* __restrict__ Gram, int n,
                                                            cplx* __restrict__ A_out,
                                                            cplx* __restrict__ MU,
                                                            cplx* __restrict__ MX,
                                                            cplx* __restrict__ Z, int p, int chol,
                                                            int* __restrict__ flags) {
  extern __shared__ cplx sm[];
  const int m = 2 * n;
  // LDS: [A][G00][UW][WW] then K (2n x 2n) and B (2n x n); Gxx and T1 live
  // inside the K region until K is formed.  Peak 10 n^2 complex.
  cplx* A = sm;                // U0^* xi
  cplx* G00 = A + n * n;       // U0^* U0
  cplx* UW = G00 + n * n;      // U0^* W
  cplx* WW = UW + n * n;       // W^* W
  cplx* K = WW + n * n;        // 2n x 2n
  cplx* B = K + m * m;         // 2n x n
  cplx* Gxx = K;               // xi^* xi   (phase 1 only)
  cplx* T1 = K + n * n;        // scratch  (phase 1 only)
  __shared__ int piv;
  cplx* Zs = sm + 18 * n * n;  // n x p, chol with Z only; loaded now, used last
  const bool zlds = n * p <= DENSE_Z_LDS;
  if (chol && Z && zlds)
    for (int t = threadIdx.x; t < n * p; t += blockDim.x) Zs[t] = Z[t];
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int a = t % n, b = t / n;
    G00[t] = Gram[b * m + a];
    A[t] = Gram[(n + b) * m + a];
    Gxx[t] = Gram[(n + b) * m + n + a];
  }
  __syncthreads();
  // U0^* W = A - G00 A / 2
  bk_matmul(T1, G00, 0, A, 0, n, n, n);
  // and, in the same phase, W^* W = Gxx - A^* A + A^* G00 A / 4 (products
  // entry by entry in the order of bk_matmul)
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t % n, j = t / n;
    UW[t] = csub(A[t], cscale(T1[t], 0.5));
    cplx agA = mk(0.0, 0.0), aa = mk(0.0, 0.0);
    for (int q = 0; q < n; ++q) {
      const cplx ac = cconj(A[i * n + q]);
      cfma(agA, ac, T1[j * n + q]);
      cfma(aa, ac, A[j * n + q]);
    }
    WW[t] = cadd(csub(Gxx[t], aa), cscale(agA, 0.25));
  }
  __syncthreads();
  // K = I - Rc^* Lc / 2,  Rc^* Lc = [[U0^*W, -U0^*U0], [W^*W, -W^*U0]]
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
    int r = t % m, c = t / m;
    cplx v;
    if (r < n && c < n) v = UW[c * n + r];
    else if (r < n) v = cscale(G00[(c - n) * n + r], -1.0);
    else if (c < n) v = WW[c * n + (r - n)];
    else v = cscale(cconj(UW[(r - n) * n + (c - n)]), -1.0);  // -(U0^*W)^*
    v = cscale(v, -0.5);
    if (r == c) v.re += 1.0;
    K[t] = v;
  }
  // B = Rc^* U0 = [G00; W^* U0] = [G00; (U0^* W)^*]
  for (int t = threadIdx.x; t < m * n; t += blockDim.x) {
    int r = t % m, c = t / m;
    B[c * m + r] = (r < n) ? G00[c * n + r] : cconj(UW[(r - n) * n + c]);
  }
  __syncthreads();
  if (bk_lu_solve(K, m, B, n, &piv)) {
    if (threadIdx.x == 0 && flags) flags[0] |= 1;
    return;
  }
  // MU = I - Y2 - A Y1 / 2,  MX = Y1   (UW and WW are free again)
  cplx* Y1 = UW;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int r = t % n, c = t / n;
    if (!chol) MX[t] = B[c * m + r];
    Y1[t] = B[c * m + r];
  }
  __syncthreads();
  bk_matmul(WW, A, 0, Y1, 0, n, n, n);  // A Y1
  // [MU; MX] (2n x n) kept in LDS past the end of B for the Cholesky pass
  cplx* Wm = B + m * n;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int r = t % n, c = t / n;
    cplx v = cscale(B[c * m + n + r], -1.0);
    v = csub(v, cscale(WW[t], 0.5));
    if (r == c) v.re += 1.0;
    if (A_out) A_out[t] = A[t];
    if (chol) {
      Wm[c * m + r] = v;
      Wm[c * m + n + r] = B[c * m + r];
    } else {
      MU[t] = v;
    }
  }
  if (!chol) return;
  // G1 = W^* (Gram W), W = [MU; MX]; the Gram again from memory
  cplx* Gs = Wm + m * n;  // 2n x 2n region: G1, then R and R^{-1} beside it
  cplx* T = Gs + m * m;   // 2n x n
  cplx* R = Gs + n * n;
  cplx* Ri = R + n * n;
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) Gs[t] = Gram[t];
  __syncthreads();
  bk_matmul(T, Gs, 0, Wm, 0, m, m, n);
  bk_matmul(Gs, Wm, 1, T, 0, n, m, n);
  if (bk_chol(Gs, R, n, 0.0)) {
    if (threadIdx.x == 0 && flags) atomicOr(&flags[0], 2);
    return;
  }
  bk_triu_inv(R, Ri, n);
  bk_matmul(T, Wm, 0, Ri, 0, m, n, n);  // [MU; MX] R^{-1}
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int r = t % n, c = t / n;
    MU[t] = T[c * m + r];
    MX[t] = T[c * m + n + r];
  }
  if (Z && zlds) {
    // Z <- R Z from the copy in LDS, one entry per thread (R upper triangular)
    for (int t = threadIdx.x; t < n * p; t += blockDim.x) {
      const int a = t % n, i = t / n;
      cplx sz = mk(0.0, 0.0);
      for (int b = a; b < n; ++b) cfma(sz, R[b * n + a], Zs[i * n + b]);
      Z[t] = sz;
    }
  } else if (Z) {
    // the same products column by column in place (a column is read before
    // it is written; R is upper triangular, so entry a needs rows b >= a)
    for (int i = threadIdx.x; i < p; i += blockDim.x) {
      cplx* zc = Z + (size_t)i * n;
      for (int a = 0; a < n; ++a) {
        cplx sz = mk(0.0, 0.0);
        for (int b = a; b < n; ++b) cfma(sz, R[b * n + a], zc[b]);
        zc[a] = sz;
      }
    }
  }
}

// Tangent velocity, first half.  Input A = U0^* xi and
// Gram2 = [U0, xi]^* [X, Ux] (2n x 2n): U0^*X = B1, U0^*Ux = C0x, xi^*X.
// W^* X = xi^* X - A^* B1 / 2;  Minv = (U0^* Ux + I)^{-1};
// Ups = (2 X - W B1 + U0 (W^* X)) Minv
//     = X (2 Minv) + xi (-B1 Minv) + U0 ((A B1 / 2 + W^* X) Minv).
__global__ void __launch_bounds__(DTPB) dense_tangent1_kernel(const cplx* __restrict__ Ag,
                                                              const cplx* __restrict__ Gram2,
                                                              int n, cplx* __restrict__ M1,
                                                              cplx* __restrict__ M2,
                                                              cplx* __restrict__ M3,
                                                              cplx* __restrict__ C0x_out,
                                                              int* __restrict__ flags) {
  extern __shared__ cplx sm[];
  const int m = 2 * n;
  cplx* A = sm;
  cplx* B1 = A + n * n;
  cplx* C0x = B1 + n * n;
  cplx* XX = C0x + n * n;
  cplx* T1 = XX + n * n;
  cplx* T2 = T1 + n * n;
  cplx* Mi = T2 + n * n;
  __shared__ int piv;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int a = t % n, b = t / n;
    A[t] = Ag[t];
    B1[t] = Gram2[b * m + a];
    C0x[t] = Gram2[(n + b) * m + a];
    XX[t] = Gram2[b * m + n + a];
  }
  __syncthreads();
  // W^* X = XX - A^* B1 / 2  -> XX
  bk_matmul(T1, A, 1, B1, 0, n, n, n);
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) XX[t] = csub(XX[t], cscale(T1[t], 0.5));
  // Minv = (C0x + I)^{-1}
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int r = t % n, c = t / n;
    T2[t] = C0x[t];
    if (r == c) T2[t].re += 1.0;
    Mi[t] = (r == c) ? mk(1.0, 0.0) : mk(0.0, 0.0);
    if (C0x_out) C0x_out[t] = C0x[t];
  }
  __syncthreads();
  if (bk_lu_solve(T2, n, Mi, n, &piv)) {
    if (threadIdx.x == 0 && flags) flags[0] |= 1;
    return;
  }
  // M1 = 2 Minv
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) M1[t] = cscale(Mi[t], 2.0);
  // M2 = -B1 Minv
  bk_matmul(T1, B1, 0, Mi, 0, n, n, n);
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) M2[t] = cscale(T1[t], -1.0);
  __syncthreads();
  // M3 = (A B1 / 2 + W^*X) Minv
  bk_matmul(T1, A, 0, B1, 0, n, n, n);
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) T2[t] = cadd(cscale(T1[t], 0.5), XX[t]);
  __syncthreads();
  bk_matmul(T1, T2, 0, Mi, 0, n, n, n);
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) M3[t] = T1[t];
}

// Tangent velocity, second half.  Gram3 = [Ux, U0]^* Ups (2n x n): D1 = Ux^*Ups,
// D0 = U0^*Ups.  Y = Ups - U0 C with C = (Ux^* U0 + I)^{-1} (D1 + D0) + D0^*
// (Ups^* U0 = D0^*).  Output xi1 = dt Y = Ups (dt I) + U0 (-dt C).
__global__ void __launch_bounds__(DTPB) dense_tangent2_kernel(const cplx* __restrict__ Gram3,
                                                              const cplx* __restrict__ C0x, int n,
                                                              double dt, cplx* __restrict__ M1,
                                                              cplx* __restrict__ M2,
                                                              int* __restrict__ flags) {
  extern __shared__ cplx sm[];
  const int m = 2 * n;
  cplx* T = sm;          // (C0x^* + I)
  cplx* Rhs = T + n * n; // D1 + D0
  cplx* D0 = Rhs + n * n;
  __shared__ int piv;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int r = t % n, c = t / n;
    cplx d1 = Gram3[c * m + r];
    cplx d0 = Gram3[c * m + n + r];
    D0[t] = d0;
    Rhs[t] = cadd(d1, d0);
    T[t] = cconj(C0x[r * n + c]);
    if (r == c) T[t].re += 1.0;
  }
  __syncthreads();
  if (bk_lu_solve(T, n, Rhs, n, &piv)) {
    if (threadIdx.x == 0 && flags) flags[0] |= 1;
    return;
  }
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int r = t % n, c = t / n;
    cplx C = cadd(Rhs[t], cconj(D0[r * n + c]));
    M2[t] = cscale(C, -dt);
    M1[t] = (r == c) ? mk(dt, 0.0) : mk(0.0, 0.0);
  }
}

// Tangent velocity in one pass, from G4 = [U0, xi, Ux, X]^* [U0, xi, Ux, X]
// (4n x 4n; block (I, J) = the I-th list entry ^* the J-th).  The two halves
// above, with Ups = X M1 + xi M2 + U0 M3 never formed: its Grams follow from
// G4, D1 = Ux^*X M1 + Ux^*xi M2 + Ux^*U0 M3 and D0 = U0^*X M1 + U0^*xi M2 +
// U0^*U0 M3, and
//   xi1 = dt Y = X (dt M1) + xi (dt M2) + U0 (dt M3 - dt C),
//   C = (Ux^* U0 + I)^{-1} (D1 + D0) + D0^*.
// Output K1, K2, K3 (n x n) for the row combination.
__global__ void __launch_bounds__(DTPB) dense_tangent_kernel(const cplx* __restrict__ G4, int n,
                                                             double dt, cplx* __restrict__ K1,
                                                             cplx* __restrict__ K2,
                                                             cplx* __restrict__ K3,
                                                             int* __restrict__ flags) {
  extern __shared__ cplx sm[];
  const int nn = n * n, m4 = 4 * n;
  cplx* A = sm;            // U0^* xi
  cplx* B1 = A + nn;       // U0^* X
  cplx* C0x = B1 + nn;     // U0^* Ux
  cplx* XX = C0x + nn;     // xi^* X, then W^* X
  cplx* UxX = XX + nn;     // Ux^* X
  cplx* Uxxi = UxX + nn;   // Ux^* xi
  cplx* UxU0 = Uxxi + nn;  // Ux^* U0
  cplx* G00 = UxU0 + nn;   // U0^* U0
  cplx* Mi = G00 + nn;     // (C0x + I)^{-1}
  cplx* M2 = Mi + nn;
  cplx* M3 = M2 + nn;
  cplx* D1 = M3 + nn;
  cplx* D0 = D1 + nn;
  cplx* T1 = D0 + nn;
  cplx* T2 = T1 + nn;
  __shared__ int piv;
  for (int t = threadIdx.x; t < nn; t += blockDim.x) {
    const int a = t % n, b = t / n;
    auto blk = [&](int I, int J) { return G4[(size_t)(J * n + b) * m4 + I * n + a]; };
    A[t] = blk(0, 1);
    B1[t] = blk(0, 3);
    C0x[t] = blk(0, 2);
    XX[t] = blk(1, 3);
    UxX[t] = blk(2, 3);
    Uxxi[t] = blk(2, 1);
    UxU0[t] = blk(2, 0);
    G00[t] = blk(0, 0);
  }
  __syncthreads();
  // W^* X = xi^* X - A^* B1 / 2
  bk_matmul(T1, A, 1, B1, 0, n, n, n);
  for (int t = threadIdx.x; t < nn; t += blockDim.x) XX[t] = csub(XX[t], cscale(T1[t], 0.5));
  // Minv = (C0x + I)^{-1}
  for (int t = threadIdx.x; t < nn; t += blockDim.x) {
    const int r = t % n, c = t / n;
    T2[t] = C0x[t];
    if (r == c) T2[t].re += 1.0;
    Mi[t] = (r == c) ? mk(1.0, 0.0) : mk(0.0, 0.0);
  }
  __syncthreads();
  if (bk_lu_solve(T2, n, Mi, n, &piv)) {
    if (threadIdx.x == 0 && flags) flags[0] |= 1;
    return;
  }
  // M2 = -B1 Minv;  M3 = (A B1 / 2 + W^* X) Minv  (M1 = 2 Minv); products
  // formed entry by entry, independent ones in the same phase
  for (int t = threadIdx.x; t < nn; t += blockDim.x) {
    const int i = t % n, j = t / n;
    M2[t] = cscale(mm_entry(B1, Mi, i, j, n), -1.0);
    T2[t] = cadd(cscale(mm_entry(A, B1, i, j, n), 0.5), XX[t]);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nn; t += blockDim.x) M3[t] = mm_entry(T2, Mi, t % n, t / n, n);
  __syncthreads();
  // D1 = Ux^*X M1 + Ux^*xi M2 + Ux^*U0 M3;  D0 = U0^*X M1 + U0^*xi M2 + U0^*U0 M3;
  // then C = (C0x^* + I)^{-1} (D1 + D0) + D0^*  (the system in T2, the right
  // side in T1)
  for (int t = threadIdx.x; t < nn; t += blockDim.x) {
    const int r = t % n, c = t / n;
    const cplx d1 = cadd(cadd(cscale(mm_entry(UxX, Mi, r, c, n), 2.0), mm_entry(Uxxi, M2, r, c, n)),
                         mm_entry(UxU0, M3, r, c, n));
    const cplx d0 = cadd(cadd(cscale(mm_entry(B1, Mi, r, c, n), 2.0), mm_entry(A, M2, r, c, n)),
                         mm_entry(G00, M3, r, c, n));
    D0[t] = d0;
    T1[t] = cadd(d1, d0);
    cplx tv = cconj(C0x[r * n + c]);
    if (r == c) tv.re += 1.0;
    T2[t] = tv;
  }
  __syncthreads();
  if (bk_lu_solve(T2, n, T1, n, &piv)) {
    if (threadIdx.x == 0 && flags) flags[0] |= 1;
    return;
  }
  for (int t = threadIdx.x; t < nn; t += blockDim.x) {
    const int r = t % n, c = t / n;
    const cplx C = cadd(T1[t], cconj(D0[r * n + c]));
    K1[t] = cscale(Mi[t], 2.0 * dt);
    K2[t] = cscale(M2[t], dt);
    K3[t] = cscale(csub(M3[t], C), dt);
  }
}

// One Cholesky-QR pass in one launch: every block factors the n x n Gram
// U~^* U~ = R^* R itself (a few microseconds, beside its loads of U~) and
// forms R^{-1}, then U~ <- U~ R^{-1} for its rows; block 0 also writes
// Z~ <- R Z~.  Replaces a Cholesky launch followed by a row combination.
template <int MC>
__global__ void __launch_bounds__(256) cholqr_apply_kernel(const cplx* __restrict__ Gram, int n,
                                                           cplx* __restrict__ U, int N,
                                                           cplx* __restrict__ Z, int p,
                                                           int* __restrict__ flags) {
  __shared__ cplx G[MC * MC], R[MC * MC], Ri[MC * MC];
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int lc = min(l, N - 1);
  // this thread's row of U~, loaded before the factorisation
  cplx u[MC];
#pragma unroll
  for (int k = 0; k < MC; ++k) {
    const cplx v = U[(size_t)min(k, n - 1) * N + lc];
    u[k] = (k < n) ? v : mk(0.0, 0.0);
  }
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) G[t] = Gram[t];
  __syncthreads();
  if (bk_chol(G, R, n, 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && flags) atomicOr(&flags[0], 2);
    return;
  }
  bk_triu_inv(R, Ri, n);
  if (l < N) {
    // row of U~ R^{-1} (R^{-1} upper triangular)
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      if (c < n) {
        cplx sc = mk(0.0, 0.0);
#pragma unroll
        for (int k = 0; k <= c; ++k) cfma(sc, u[k], Ri[c * n + k]);
        U[(size_t)c * N + l] = sc;
      }
    }
  }
  if (blockIdx.x == 0 && Z) {
    // Z <- R Z, one column per thread (the column is read before written)
    for (int i = threadIdx.x; i < p; i += blockDim.x) {
      cplx zc[MC];
#pragma unroll
      for (int a = 0; a < MC; ++a) zc[a] = (a < n) ? Z[(size_t)i * n + a] : mk(0.0, 0.0);
#pragma unroll
      for (int a = 0; a < MC; ++a) {
        if (a < n) {
          cplx sz = mk(0.0, 0.0);
#pragma unroll
          for (int b = a; b < MC; ++b)
            if (b < n) cfma(sz, R[b * n + a], zc[b]);
          Z[(size_t)i * n + a] = sz;
        }
      }
    }
  }
}

// Fixed-point control of the implicit midpoint stage, one block per column
// i (a wavefront; lane a takes entry a).  k_new = -i g (g = gF, plus
// (C1 Z - conj(C2) conj(Z)) / 2 when the projection covered positions only:
// i U~^* V_r with V_r = Im(U~ Z~)).  For an active column:
// rel = |k_new - k| / |k_new| (squared moduli summed in entry order);
// converged if rel < tol, stalled if not converged, rel >= the previous rel
// (a particle at a node puts the map into a cycle of jumps and contraction
// steps) and the smaller of the two below stall_tol (a cycle without a
// contracted phase below that floor keeps iterating); k <- k_new;
// ZG <- Zeval; if still active, Zeval <- Z0 + dt/2 k.  counters[0] loses one
// per column that stops (it counts the active columns), counters[1] gains
// the stalled ones, counters[2] becomes the launch ordinal `iter`, and the
// double at counters + 6 is the largest rel accepted by a stall (atomic
// maximum of the bit patterns, which order like the values for rel >= 0).
// fixed != 0 disables the test.
__global__ void __launch_bounds__(64) dense_fp_update_kernel(
    const cplx* __restrict__ gF, const cplx* __restrict__ C12, int n, int p,
    const cplx* __restrict__ Z0, cplx* __restrict__ Zeval, cplx* __restrict__ ZG,
    cplx* __restrict__ k, double* __restrict__ prev, int* __restrict__ active, double dt,
    double tol, double stall_tol, int fixed, int linear_part, int iter,
    int* __restrict__ counters) {
  // nothing left to iterate: a speculative launch after convergence (a
  // column still active keeps counters[0] >= 1 until its block has run)
  if (counters[0] == 0) return;
  const int i = blockIdx.x;
  if (!active[i]) return;
  __shared__ cplx ze[32];
  __shared__ double dq[32], kq[32];
  __shared__ int go_on;
  const int a = threadIdx.x;
  if (a < n) ze[a] = Zeval[(size_t)i * n + a];
  __syncthreads();
  cplx knew = mk(0.0, 0.0);
  if (a < n) {
    const size_t t = (size_t)i * n + a;
    cplx g = gF[t];
    if (linear_part) {
      cplx sl = mk(0.0, 0.0);
      for (int b = 0; b < n; ++b) {
        cfma(sl, C12[b * n + a], ze[b]);
        cfma(sl, cscale(cconj(C12[n * n + b * n + a]), -1.0), cconj(ze[b]));
      }
      g = cadd(g, cscale(sl, 0.5));
    }
    knew = mk(g.im, -g.re);  // -i g
    const cplx d = csub(knew, k[t]);
    dq[a] = cabs2(d);
    kq[a] = cabs2(knew);
    k[t] = knew;
    ZG[t] = ze[a];
  }
  __syncthreads();
  if (a == 0) {
    double dn = 0.0, kn = 0.0;
    for (int b = 0; b < n; ++b) {
      dn += dq[b];
      kn += kq[b];
    }
    bool done = false;
    if (!fixed) {
      const double rel = (kn > 0.0) ? sqrt(dn) / sqrt(kn) : sqrt(dn);
      const double pv = prev[i];
      const bool conv = rel < tol;
      const bool stall = !conv && rel >= pv && fmin(rel, pv) < stall_tol;
      prev[i] = rel;
      done = conv || stall;
      if (stall) {
        atomicAdd(&counters[1], 1);
        atomicMax(reinterpret_cast<unsigned long long*>(counters + 6),
                  (unsigned long long)__double_as_longlong(rel));
      }
    }
    if (done) {
      active[i] = 0;
      atomicSub(&counters[0], 1);
    }
    atomicMax(&counters[2], iter);
    go_on = done ? 0 : 1;
  }
  __syncthreads();
  if (go_on && a < n) {
    const cplx z0 = Z0[(size_t)i * n + a];
    Zeval[(size_t)i * n + a] = mk(z0.re + 0.5 * dt * knew.re, z0.im + 0.5 * dt * knew.im);
  }
}

// start of a fixed-point solve: all columns active, no previous update
__global__ void fp_init_kernel(double* prev, int* active, int* counters, int p) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < p) {
    prev[t] = INFINITY;
    active[t] = 1;
  }
  // [0] columns still active (all, before the first iteration), [1] stalled
  // columns, [2] iterations that updated at least one column, [6..7] the
  // largest update accepted by a stall (a double)
  if (t < 4) counters[t] = (t == 0) ? p : 0;
  if (t == 6 || t == 7) counters[t] = 0;
}

// End of a step with the DEIM chain: the error word of the chain in flight
// (3) is folded into the step's word (2) and cleared for the next chain; the
// stop word (12) of a chain enqueued next is set when this step failed.
__global__ void fold_status_kernel(int* status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int tail = status[2] | status[3];
    status[2] = tail;
    status[3] = 0;
    status[12] = status[0] | tail;
  }
}
void launch_fold_status(hipStream_t s, int* status) {
  hipLaunchKernelGGL(fold_status_kernel, dim3(1), dim3(64), 0, s, status);
}

// Z1 = Z0 + dt k
__global__ void dense_finish_z_kernel(const cplx* __restrict__ Z0, const cplx* __restrict__ k,
                                      int n, int p, double dt, cplx* __restrict__ Z1) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * p) return;
  Z1[t] = mk(Z0[t].re + dt * k[t].re, Z0[t].im + dt * k[t].im);
}

// Hermitian eigendecomposition of an m x m matrix in global memory (A is
// overwritten, V receives eigenvectors, lam eigenvalues in decreasing order).
__global__ void __launch_bounds__(DTPB) dense_herm_eig_kernel(cplx* A, int m, cplx* V,
                                                              double* lam, int* flags) {
  extern __shared__ cplx sm[];  // 2 m^2 when m <= 64
  __shared__ cplx rot[3 * 66 + 3];
  __shared__ int pr[132];
  __shared__ double lm[128];
  cplx* As = A;
  cplx* Vs = V;
  if (m <= 64) {
    As = sm;
    Vs = sm + m * m;
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) As[t] = A[t];
    __syncthreads();
  }
  bk_jacobi(As, Vs, lm, m, rot, pr);
  if (m <= 64)
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) V[t] = Vs[t];
  for (int t = threadIdx.x; t < m; t += blockDim.x) lam[t] = lm[t];
  (void)flags;
}

// ---------------------------------------------------------------------------
// layout conversions
// ---------------------------------------------------------------------------
__global__ void fill_cplx_kernel(cplx* a, size_t n, cplx v) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) a[t] = v;
}
__global__ void copy_cplx_kernel(cplx* dst, const cplx* src, size_t n) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[t];
}
__global__ void make_complex_kernel(const double* X, const double* V, size_t n, cplx* C) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) C[t] = mk(X[t], V[t]);
}
__global__ void split_complex_kernel(const cplx* C, size_t n, double* X, double* V) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    if (X) X[t] = C[t].re;
    if (V) V[t] = C[t].im;
  }
}
// U_X = [A, -B] (N x 2n, ld N) from U~ = A + iB
__global__ void ux_from_u_kernel(const cplx* U, int N, int n, double* UX) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t tot = (size_t)N * n;
  if (t >= tot) return;
  cplx u = U[t];
  UX[t] = u.re;
  UX[tot + t] = -u.im;
}
__global__ void u_from_ux_kernel(const double* UX, int N, int n, cplx* U) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t tot = (size_t)N * n;
  if (t >= tot) return;
  U[t] = mk(UX[t], -UX[tot + t]);
}
// Z~ = Z_q + i Z_p (n x p, ld n) from real Z (2n x p, ld 2n)
__global__ void z_from_real_kernel(const double* Z, int n, int p, cplx* Zc) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * p) return;
  int a = t % n, i = t / n;
  Zc[t] = mk(Z[(size_t)i * 2 * n + a], Z[(size_t)i * 2 * n + n + a]);
}
__global__ void z_to_real_kernel(const cplx* Zc, int n, int p, double* Z) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * p) return;
  int a = t % n, i = t / n;
  Z[(size_t)i * 2 * n + a] = Zc[t].re;
  Z[(size_t)i * 2 * n + n + a] = Zc[t].im;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(size_t n) { return (unsigned)((n + 255) / 256); }

// Kernels whose work is a chain of small steps separated by block barriers
// run as one wavefront for small ranks (its barriers cost next to nothing);
// larger ranks use four wavefronts.
static int dense_chain_threads(int n) { return (n <= 8) ? 64 : DTPB; }

void launch_dense_spinv(hipStream_t s, const cplx* Z, int n, int p, double rtol, cplx* Q,
                        double* sigma2, int* flags) {
  const size_t sh = (size_t)((n * p <= DENSE_Z_LDS ? n * p : 0) + 3 * n * n) * sizeof(cplx);
  ALLOW_BIG_LDS(dense_spinv_kernel);
  hipLaunchKernelGGL(dense_spinv_kernel, dim3(1), dim3(dense_chain_threads(n)), sh, s, Z, n, p,
                     rtol, Q, sigma2, flags);
}
void launch_dense_xfinish(hipStream_t s, const cplx* g, const cplx* Q, int n, int p, double dt,
                          cplx* k1, cplx* MP, cplx* MU) {
  const size_t sh = (n * p <= DENSE_Z_LDS) ? (size_t)(2 * n * p) * sizeof(cplx) : 0;
  ALLOW_BIG_LDS(dense_xfinish_kernel);
  hipLaunchKernelGGL(dense_xfinish_kernel, dim3(1), dim3(DTPB), sh, s, g, Q, n, p, dt, k1, MP,
                     MU);
}
void launch_dense_cayley(hipStream_t s, const cplx* Gram, int n, cplx* A_out, cplx* MU,
                         cplx* MX, int* flags, bool chol, cplx* Z, int p) {
  // 10 n^2 for the solve; with chol, W (2 n^2), the Gram (4 n^2), T (2 n^2)
  // and Z (n p)
  size_t sh = (size_t)((chol ? 18 : 10) * n * n + (chol && Z && n * p <= DENSE_Z_LDS ? n * p : 0)) *
              sizeof(cplx);
  ALLOW_BIG_LDS(dense_cayley_kernel);
  hipLaunchKernelGGL(dense_cayley_kernel, dim3(1), dim3(dense_chain_threads(n)), sh, s, Gram, n,
                     A_out, MU, MX, Z, p, (int)chol, flags);
}
void launch_dense_tangent1(hipStream_t s, const cplx* A, const cplx* Gram2, int n, cplx* M1,
                           cplx* M2, cplx* M3, cplx* C0x_out, int* flags) {
  size_t sh = (size_t)7 * n * n * sizeof(cplx);
  ALLOW_BIG_LDS(dense_tangent1_kernel);
  hipLaunchKernelGGL(dense_tangent1_kernel, dim3(1), dim3(dense_chain_threads(n)), sh, s, A, Gram2,
                     n, M1, M2, M3, C0x_out, flags);
}
void launch_dense_tangent2(hipStream_t s, const cplx* Gram3, const cplx* C0x, int n, double dt,
                           cplx* M1, cplx* M2, int* flags) {
  size_t sh = (size_t)3 * n * n * sizeof(cplx);
  hipLaunchKernelGGL(dense_tangent2_kernel, dim3(1), dim3(dense_chain_threads(n)), sh, s, Gram3,
                     C0x, n, dt, M1, M2, flags);
}
void launch_dense_tangent(hipStream_t s, const cplx* G4, int n, double dt, cplx* K1, cplx* K2,
                          cplx* K3, int* flags) {
  const size_t sh = (size_t)15 * n * n * sizeof(cplx);
  ALLOW_BIG_LDS(dense_tangent_kernel);
  hipLaunchKernelGGL(dense_tangent_kernel, dim3(1), dim3(dense_chain_threads(n)), sh, s, G4, n, dt,
                     K1, K2, K3, flags);
}
void launch_cholqr_apply(hipStream_t s, const cplx* Gram, int n, cplx* U, int N, cplx* Z, int p,
                         int* flags) {
  dim3 grid((N + 255) / 256);
  if (n <= 8)
    hipLaunchKernelGGL(cholqr_apply_kernel<8>, grid, dim3(256), 0, s, Gram, n, U, N, Z, p, flags);
  else if (n <= 16)
    hipLaunchKernelGGL(cholqr_apply_kernel<16>, grid, dim3(256), 0, s, Gram, n, U, N, Z, p, flags);
  else
    hipLaunchKernelGGL(cholqr_apply_kernel<32>, grid, dim3(256), 0, s, Gram, n, U, N, Z, p, flags);
}
void launch_dense_fp_update(hipStream_t s, const cplx* gF, const cplx* C12, int n, int p,
                            const cplx* Z0, cplx* Zeval, cplx* ZG, cplx* k, double* prev,
                            int* active, double dt, double tol, double stall_tol, int fixed,
                            int linear_part, int iter, int* counters) {
  hipLaunchKernelGGL(dense_fp_update_kernel, dim3(p), dim3(64), 0, s, gF, C12, n, p, Z0, Zeval,
                     ZG, k, prev, active, dt, tol, stall_tol, fixed, linear_part, iter, counters);
}
void launch_dense_finish_z(hipStream_t s, const cplx* Z0, const cplx* k, int n, int p, double dt,
                           cplx* Z1) {
  hipLaunchKernelGGL(dense_finish_z_kernel, dim3(nblk((size_t)n * p)), dim3(256), 0, s, Z0, k, n,
                     p, dt, Z1);
}
void launch_fp_init(hipStream_t s, double* prev, int* active, int* counters, int p) {
  hipLaunchKernelGGL(fp_init_kernel, dim3(nblk((size_t)(p > 4 ? p : 4))), dim3(256), 0, s, prev,
                     active, counters, p);
}
void launch_dense_herm_eig(hipStream_t s, cplx* A, int m, cplx* V, double* lam, int* flags) {
  size_t sh = (m <= 64) ? (size_t)2 * m * m * sizeof(cplx) : 0;
  ALLOW_BIG_LDS(dense_herm_eig_kernel);
  hipLaunchKernelGGL(dense_herm_eig_kernel, dim3(1), dim3(DTPB), sh, s, A, m, V, lam, flags);
}
void launch_fill_cplx(hipStream_t s, cplx* a, size_t n, cplx v) {
  if (n) hipLaunchKernelGGL(fill_cplx_kernel, dim3(nblk(n)), dim3(256), 0, s, a, n, v);
}
void launch_copy_cplx(hipStream_t s, cplx* dst, const cplx* src, size_t n) {
  if (n) hipLaunchKernelGGL(copy_cplx_kernel, dim3(nblk(n)), dim3(256), 0, s, dst, src, n);
}
void launch_make_complex(hipStream_t s, const double* X, const double* V, size_t n, cplx* C) {
  hipLaunchKernelGGL(make_complex_kernel, dim3(nblk(n)), dim3(256), 0, s, X, V, n, C);
}
void launch_split_complex(hipStream_t s, const cplx* C, size_t n, double* X, double* V) {
  hipLaunchKernelGGL(split_complex_kernel, dim3(nblk(n)), dim3(256), 0, s, C, n, X, V);
}
void launch_ux_from_u(hipStream_t s, const cplx* U, int N, int n, double* UX) {
  hipLaunchKernelGGL(ux_from_u_kernel, dim3(nblk((size_t)N * n)), dim3(256), 0, s, U, N, n, UX);
}
void launch_u_from_ux(hipStream_t s, const double* UX, int N, int n, cplx* U) {
  hipLaunchKernelGGL(u_from_ux_kernel, dim3(nblk((size_t)N * n)), dim3(256), 0, s, UX, N, n, U);
}
void launch_z_from_real(hipStream_t s, const double* Z, int n, int p, cplx* Zc) {
  hipLaunchKernelGGL(z_from_real_kernel, dim3(nblk((size_t)n * p)), dim3(256), 0, s, Z, n, p, Zc);
}
void launch_z_to_real(hipStream_t s, const cplx* Zc, int n, int p, double* Z) {
  hipLaunchKernelGGL(z_to_real_kernel, dim3(nblk((size_t)n * p)), dim3(256), 0, s, Zc, n, p, Z);
}

// ---------------------------------------------------------------------------
// rank adaptation
// ---------------------------------------------------------------------------

// Gp <- Gp - g^* g  (Gp = G~^* G~, p x p; g = U~^* G~, n x p), i.e. H^* H for
// H = (I - U~ U~^*) G~; eps = sqrt(1 - ||g||^2 / ||G||^2) (the rank indicator,
// ||(I - U U^T) J G|| / ||G|| with U^T J = J U^T).
__global__ void __launch_bounds__(DTPB) dense_hh_kernel(cplx* __restrict__ Gp,
                                                        const cplx* __restrict__ g, int n, int p,
                                                        double* __restrict__ eps_out) {
  __shared__ double red[DTPB / 64];
  double tr = 0.0, gn = 0.0;
  for (int i = threadIdx.x; i < p; i += blockDim.x) tr += Gp[i * p + i].re;
  for (int t = threadIdx.x; t < n * p; t += blockDim.x) gn += cabs2(g[t]);
  tr = block_sum(tr, red);
  gn = block_sum(gn, red);
  for (int t = threadIdx.x; t < p * p; t += blockDim.x) {
    int i = t % p, j = t / p;
    cplx s = Gp[t];
    for (int k = 0; k < n; ++k) s = csub(s, cmulc(g[(size_t)i * n + k], g[(size_t)j * n + k]));
    Gp[t] = s;
  }
  if (threadIdx.x == 0 && eps_out) *eps_out = (tr > 0.0) ? sqrt(fmax(0.0, 1.0 - gn / tr)) : 0.0;
}

// W[:, j] = V[:, j] / sqrt(lam_j) (p x k) and T = -g W (n x k): the new basis
// vectors are y_j = H w_j / sigma_j = G~ W[:, j] + U~ T[:, j].
__global__ void __launch_bounds__(DTPB) dense_grow_prep_kernel(
    const cplx* __restrict__ V, const double* __restrict__ lam, const cplx* __restrict__ g, int n,
    int p, int k, cplx* __restrict__ W, cplx* __restrict__ T, int* __restrict__ flags) {
  for (int t = threadIdx.x; t < p * k; t += blockDim.x) {
    int j = t / p;
    double l = lam[j];
    if (!(l > 0.0)) {
      if (flags) flags[0] |= 4;
      W[t] = mk(0.0, 0.0);
    } else {
      W[t] = cscale(V[t], 1.0 / sqrt(l));
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n * k; t += blockDim.x) {
    int a = t % n, j = t / n;
    cplx s = mk(0.0, 0.0);
    for (int i = 0; i < p; ++i) cfma(s, g[(size_t)i * n + a], W[(size_t)j * p + i]);
    T[t] = cscale(s, -1.0);
  }
}

// Canonical phase of columns col0 .. col0+k-1 of U (N rows): the entry of
// largest modulus (smallest row index on ties) is made real positive.
// One block per column.
__global__ void __launch_bounds__(1024) colphase_kernel(cplx* __restrict__ U, int N, int col0) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  cplx* u = U + (size_t)(col0 + blockIdx.x) * N;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int l = threadIdx.x; l < N; l += blockDim.x) {
    double a = cabs2(u[l]);
    if (a > best) {
      best = a;
      bi = l;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      double a = sv[threadIdx.x + o];
      int ai = si[threadIdx.x + o];
      if (a > sv[threadIdx.x] || (a == sv[threadIdx.x] && ai < si[threadIdx.x])) {
        sv[threadIdx.x] = a;
        si[threadIdx.x] = ai;
      }
    }
    __syncthreads();
  }
  const cplx a = u[si[0]];
  const double m = sqrt(cabs2(a));
  const cplx ph = (m > 0.0) ? mk(a.re / m, -a.im / m) : mk(1.0, 0.0);
  __syncthreads();
  for (int l = threadIdx.x; l < N; l += blockDim.x) u[l] = cmul(u[l], ph);
}

// Zout (nout x p) from Zin (nin x p): copy the common rows, zero the rest.
__global__ void z_resize_kernel(const cplx* __restrict__ Zin, int nin, cplx* __restrict__ Zout,
                                int nout, int p) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nout * p) return;
  int a = t % nout, i = t / nout;
  Zout[t] = (a < nin) ? Zin[(size_t)i * nin + a] : mk(0.0, 0.0);
}

// Shrink: eigendecomposition Z~ Z~^* = V diag(sigma^2) V^* (decreasing, each
// column of V with canonical phase), V (n x n) and Znew = V^* Z~ (n x p).
__global__ void __launch_bounds__(DTPB) dense_shrink_kernel(const cplx* __restrict__ Z, int n,
                                                            int p, cplx* __restrict__ Vout,
                                                            cplx* __restrict__ Znew,
                                                            double* __restrict__ sig2) {
  __shared__ cplx S[32 * 32];
  __shared__ cplx V[32 * 32];
  __shared__ cplx rot[3 * 17 + 3];
  __shared__ int pr[40];
  __shared__ double lam[32];
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int a = t % n, b = t / n;
    cplx s = mk(0.0, 0.0);
    for (int i = 0; i < p; ++i) cfma(s, Z[(size_t)i * n + a], cconj(Z[(size_t)i * n + b]));
    S[t] = s;
  }
  __syncthreads();
  bk_jacobi(S, V, lam, n, rot, pr);
  // canonical phase of each eigenvector
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    int bi = 0;
    double bv = -1.0;
    for (int r = 0; r < n; ++r) {
      double a = cabs2(V[c * n + r]);
      if (a > bv) {
        bv = a;
        bi = r;
      }
    }
    cplx a = V[c * n + bi];
    double m = sqrt(cabs2(a));
    cplx ph = (m > 0.0) ? mk(a.re / m, -a.im / m) : mk(1.0, 0.0);
    for (int r = 0; r < n; ++r) V[c * n + r] = cmul(V[c * n + r], ph);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) Vout[t] = V[t];
  for (int t = threadIdx.x; t < n * p; t += blockDim.x) {
    int a = t % n, i = t / n;
    cplx s = mk(0.0, 0.0);
    for (int b = 0; b < n; ++b) cfmac(s, V[a * n + b], Z[(size_t)i * n + b]);
    Znew[t] = s;
  }
  if (sig2)
    for (int t = threadIdx.x; t < n; t += blockDim.x) sig2[t] = lam[t];
}

void launch_dense_hh(hipStream_t s, cplx* Gp, const cplx* g, int n, int p, double* eps) {
  hipLaunchKernelGGL(dense_hh_kernel, dim3(1), dim3(DTPB), 0, s, Gp, g, n, p, eps);
}
void launch_dense_grow_prep(hipStream_t s, const cplx* V, const double* lam, const cplx* g, int n,
                            int p, int k, cplx* W, cplx* T, int* flags) {
  hipLaunchKernelGGL(dense_grow_prep_kernel, dim3(1), dim3(DTPB), 0, s, V, lam, g, n, p, k, W, T,
                     flags);
}
void launch_colphase(hipStream_t s, cplx* U, int N, int col0, int k) {
  hipLaunchKernelGGL(colphase_kernel, dim3(k), dim3(1024), 0, s, U, N, col0);
}
void launch_z_resize(hipStream_t s, const cplx* Zin, int nin, cplx* Zout, int nout, int p) {
  hipLaunchKernelGGL(z_resize_kernel, dim3(nblk((size_t)nout * p)), dim3(256), 0, s, Zin, nin,
                     Zout, nout, p);
}
void launch_dense_shrink(hipStream_t s, const cplx* Z, int n, int p, cplx* V, cplx* Znew,
                         double* sig2) {
  hipLaunchKernelGGL(dense_shrink_kernel, dim3(1), dim3(DTPB), 0, s, Z, n, p, V, Znew, sig2);
}

// ---------------------------------------------------------------------------
// DEIM (Sec. 4.2.2): basis coefficients, greedy selection and weights
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Real symmetric eigendecomposition (n <= 64) in one wavefront: Householder
// reduction to tridiagonal form, accumulation of the reflectors, then the
// implicit QL iteration with Wilkinson-type shifts on the tridiagonal matrix.
// Lane r owns row r of the matrices, so every Givens rotation of the QL
// sweep is applied by each lane to its own row without barriers; the scalar
// recurrence runs redundantly on all lanes with d, e shared in LDS.
// Input: the real part of G (n x n, column-major).  Output: eigenvalues lam
// in decreasing order and eigenvectors V (n x n, column-major, real).
// ---------------------------------------------------------------------------
#define SE_LD 65
__global__ void __launch_bounds__(64) dense_symeig_kernel(const cplx* __restrict__ G, int n,
                                                          double* __restrict__ V,
                                                          double* __restrict__ lam,
                                                          int* __restrict__ flags) {
  __shared__ double A[64 * SE_LD];
  __shared__ double Z[64 * SE_LD];
  __shared__ double H[64 * SE_LD];  // Householder vectors, row k holds v_k
  __shared__ double tau[64];
  __shared__ double wv[64];
  __shared__ double dd[64];
  __shared__ double ee[64];
  __shared__ int perm[64];
  const int r = threadIdx.x;
  auto wsum = [](double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
  };
  if (r < n)
    for (int c = 0; c < n; ++c) A[r * SE_LD + c] = G[(size_t)c * n + r].re;
  __syncthreads();
  // 1. Householder tridiagonalisation: H_k = I - tau_k v_k v_k^T zeroes column k
  //    below the subdiagonal; B <- H B H via p = tau B v, w = p - (tau/2 v.p) v
  for (int k = 0; k + 2 < n; ++k) {
    const double xr = (r > k && r < n) ? A[r * SE_LD + k] : 0.0;
    const double sig = wsum(xr * xr);
    const double x0 = A[(k + 1) * SE_LD + k];
    double t = 0.0, alpha = 0.0;
    if (sig > 0.0) {
      alpha = (x0 >= 0.0) ? -sqrt(sig) : sqrt(sig);
      const double vn2 = 2.0 * sig - 2.0 * alpha * x0;
      t = (vn2 > 0.0) ? 2.0 / vn2 : 0.0;
    }
    const double vr = (r > k && r < n) ? (r == k + 1 ? xr - alpha : xr) : 0.0;
    if (r < 64) H[k * SE_LD + r] = vr;
    if (r == 0) tau[k] = t;
    __syncthreads();
    if (t != 0.0) {
      double pa[4] = {0.0, 0.0, 0.0, 0.0};
      if (r > k && r < n) {
        const double* ar = A + r * SE_LD;
        const double* hv = H + k * SE_LD;
#pragma unroll 4
        for (int j = k + 1; j < n; ++j) pa[j & 3] = fma(ar[j], hv[j], pa[j & 3]);
      }
      double pr_ = t * ((pa[0] + pa[1]) + (pa[2] + pa[3]));
      const double K = 0.5 * t * wsum(vr * pr_);
      const double wr = pr_ - K * vr;
      wv[r] = wr;
      __syncthreads();
      if (r > k && r < n) {
        double* ar = A + r * SE_LD;
        const double* hv = H + k * SE_LD;
#pragma unroll 8
        for (int j = k + 1; j < n; ++j) ar[j] -= vr * wv[j] + wr * hv[j];
      }
      __syncthreads();
      if (r > k + 1 && r < n) {
        A[r * SE_LD + k] = 0.0;
        A[k * SE_LD + r] = 0.0;
      }
      if (r == 0) {
        A[(k + 1) * SE_LD + k] = alpha;
        A[k * SE_LD + k + 1] = alpha;
      }
    }
    __syncthreads();
  }
  // 2. Z = H_0 H_1 ... H_{n-3}, applied right to left to the identity
  if (r < n)
    for (int c = 0; c < n; ++c) Z[r * SE_LD + c] = (r == c) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const double t = tau[k];
    if (t == 0.0) continue;
    // s_c = v^T Z[:, c] (lane c), then Z[i, c] -= t v_i s_c (lane i)
    double sa[4] = {0.0, 0.0, 0.0, 0.0};
    if (r < n) {
      const double* hv = H + k * SE_LD;
#pragma unroll 4
      for (int i = k + 1; i < n; ++i) sa[i & 3] = fma(hv[i], Z[i * SE_LD + r], sa[i & 3]);
    }
    wv[r] = (sa[0] + sa[1]) + (sa[2] + sa[3]);
    __syncthreads();
    if (r > k && r < n) {
      const double tv = t * H[k * SE_LD + r];
      double* zr = Z + r * SE_LD;
#pragma unroll 8
      for (int c = 0; c < n; ++c) zr[c] -= tv * wv[c];
    }
    __syncthreads();
  }
  // 3. implicit QL on the tridiagonal (d, e).  Lane 0 runs the scalar
  //    recurrence of one QL iteration and records its Givens rotations
  //    (applied to columns i, i+1 for i = m-1 .. l); then every lane applies
  //    them, in order, to its own row of Z.
  double* rc = H;                 // rotation cosines (H is free now)
  double* rs = H + 64;            // rotation sines
  __shared__ int qctl[4];         // [0] l, [1] m, [2] rotations recorded, [3] state
  if (r < n) {
    dd[r] = A[r * SE_LD + r];
    ee[r] = (r + 1 < n) ? A[(r + 1) * SE_LD + r] : 0.0;
  }
  if (r == 0) {
    qctl[0] = 0;
    qctl[3] = 0;  // 0 running, 1 done, 2 iteration cap exceeded
  }
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  int iter_l = 0;  // lane 0: QL iterations spent on the current l
  for (;;) {
    if (r == 0) {
      int l = qctl[0];
      int nrec = 0, mfound = l;
      for (;;) {
        if (l >= n) {
          qctl[3] = 1;
          break;
        }
        int m = l;
        while (m < n - 1 && !(fabs(ee[m]) <= eps * (fabs(dd[m]) + fabs(dd[m + 1])))) ++m;
        if (m == l) {
          ++l;
          iter_l = 0;
          continue;
        }
        if (++iter_l > 60) {
          qctl[3] = 2;
          break;
        }
        mfound = m;
        double g = (dd[l + 1] - dd[l]) / (2.0 * ee[l]);
        double rr = hypot(g, 1.0);
        g = dd[m] - dd[l] + ee[l] / (g + (g >= 0.0 ? rr : -rr));
        double s = 1.0, c = 1.0, pp = 0.0;
        bool early = false;
        // d_{i+1} is carried in a register; e_i and d_i of the next index are
        // loaded one iteration ahead (the iteration writes index i+1 only)
        double d_up = dd[m];
        double e_i = ee[m - 1], d_i = dd[m - 1];
        for (int i = m - 1; i >= l; --i) {
          const double e_nx = (i > l) ? ee[i - 1] : 0.0;
          const double d_nx = (i > l) ? dd[i - 1] : 0.0;
          const double f = s * e_i;
          const double b = c * e_i;
          rr = hypot(f, g);
          ee[i + 1] = rr;
          if (rr == 0.0) {
            dd[i + 1] = d_up - pp;
            ee[m] = 0.0;
            early = true;
            break;
          }
          const double inv = 1.0 / rr;
          s = f * inv;
          c = g * inv;
          g = d_up - pp;
          rr = (d_i - g) * s + 2.0 * c * b;
          pp = s * rr;
          dd[i + 1] = g + pp;
          g = c * rr - b;
          rc[nrec] = c;
          rs[nrec] = s;
          ++nrec;
          d_up = d_i;
          e_i = e_nx;
          d_i = d_nx;
        }
        if (!early) {
          dd[l] -= pp;
          ee[l] = g;
          ee[m] = 0.0;
        }
        break;
      }
      qctl[0] = l;
      qctl[1] = mfound;
      qctl[2] = nrec;
    }
    __syncthreads();
    if (qctl[3] != 0) break;
    const int nrec = qctl[2];
    const int m = qctl[1];
    if (r < n && nrec > 0) {
      // rotation t acts on columns (i, i+1), i = m-1-t; the updated column i
      // is the upper operand of the next rotation, so it stays in a register
      double* zr = Z + r * SE_LD;
      double hi = zr[m];
      for (int t = 0; t < nrec; ++t) {
        const int i = m - 1 - t;
        const double lo = zr[i];
        const double c = rc[t], s = rs[t];
        zr[i + 1] = s * lo + c * hi;
        hi = c * lo - s * hi;
      }
      zr[m - nrec] = hi;
    }
    __syncthreads();
  }
  const int bad = (qctl[3] == 2);
  // 4. decreasing order
  if (r == 0) {
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int i = 0; i < n; ++i) {
      int b = i;
      for (int j = i + 1; j < n; ++j)
        if (dd[perm[j]] > dd[perm[b]]) b = j;
      int tp = perm[i];
      perm[i] = perm[b];
      perm[b] = tp;
    }
  }
  __syncthreads();
  if (r < n) {
    lam[r] = dd[perm[r]];
    for (int c = 0; c < n; ++c) V[(size_t)c * n + r] = Z[r * SE_LD + perm[c]];
  }
  if (r == 0 && bad && flags) flags[0] |= 32;
}

void launch_dense_symeig(hipStream_t s, const cplx* G, int n, double* V, double* lam, int* flags) {
  hipLaunchKernelGGL(dense_symeig_kernel, dim3(1), dim3(64), 0, s, G, n, V, lam, flags);
}

// Rank indicator from column sums of squares of G~ (p) and g (n x p):
// eps = sqrt(1 - ||g||^2 / ||G||^2).
__global__ void __launch_bounds__(DTPB) dense_indicator_kernel(const double* __restrict__ colsq,
                                                               const cplx* __restrict__ g, int n,
                                                               int p, double* __restrict__ eps_out) {
  __shared__ double red[DTPB / 64];
  double tr = 0.0, gn = 0.0;
  for (int i = threadIdx.x; i < p; i += blockDim.x) tr += colsq[i];
  for (int t = threadIdx.x; t < n * p; t += blockDim.x) gn += cabs2(g[t]);
  tr = block_sum(tr, red);
  gn = block_sum(gn, red);
  if (threadIdx.x == 0) *eps_out = (tr > 0.0) ? sqrt(fmax(0.0, 1.0 - gn / tr)) : 0.0;
}
void launch_dense_indicator(hipStream_t s, const double* colsq, const cplx* g, int n, int p,
                            double* eps) {
  hipLaunchKernelGGL(dense_indicator_kernel, dim3(1), dim3(DTPB), 0, s, colsq, g, n, p, eps);
}

// ---------------------------------------------------------------------------
// Automatic shrink (rank adaptation): the pairs whose singular value of Z~
// falls below rank_tol_down times the largest are dropped.
//
// Certificate: S~ = Z~ Z~^* (n x n); if S~ - c trace(S~) I admits a Cholesky
// factor then lambda_min(S~) > c trace(S~) >= c lambda_max (up to the
// factorisation's backward error, about n eps trace, far below c >= 1e-13),
// so sigma_min / sigma_max > sqrt(c) and, with c >= tol^2, nothing is
// dropped.  *word = 0 when certified, 1 otherwise (the singular values are
// then computed accurately by dense_zsvals_kernel).  Requires n <= 32.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(DTPB) dense_rank_cert_kernel(const cplx* __restrict__ Z, int n,
                                                               int p, double c,
                                                               int* __restrict__ word) {
  __shared__ cplx S[32 * 32];
  __shared__ cplx R[32 * 32];
  __shared__ double trs;
  extern __shared__ cplx zs[];  // Z~ (n x p) when it fits, see the launcher
  const bool lds = n * p <= 4096;
  if (lds) {
    for (int t = threadIdx.x; t < n * p; t += blockDim.x) zs[t] = Z[t];
    __syncthreads();
  }
  const cplx* Zr = lds ? zs : Z;
  // entry (a, b) of Z~ Z~^* by a group of 8 lanes (parameters strided),
  // summed by a fixed butterfly
  const int g = threadIdx.x >> 3, gl = threadIdx.x & 7;
  for (int t = g; t < n * n; t += blockDim.x >> 3) {
    const int a = t % n, b = t / n;
    cplx acc = mk(0.0, 0.0);
    for (int i = gl; i < p; i += 8) cfma(acc, Zr[(size_t)i * n + a], cconj(Zr[(size_t)i * n + b]));
    for (int o = 4; o > 0; o >>= 1) {
      acc.re += __shfl_xor(acc.re, o, 8);
      acc.im += __shfl_xor(acc.im, o, 8);
    }
    if (gl == 0) S[t] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int a = 0; a < n; ++a) tr += S[a * n + a].re;
    trs = tr;
  }
  __syncthreads();
  const int bad = (trs > 0.0) ? bk_chol(S, R, n, c * trs) : 1;
  if (threadIdx.x == 0) *word = bad ? 1 : 0;
}

// Singular values of Z~ (n x p) by one-sided Jacobi on its rows (high
// relative accuracy; no Gram is formed): pairs of rows are rotated until
// every pair is orthogonal to 1e-15 of the product of their norms; the
// singular values are then the row norms.  The rows are copied to `work`
// (n x p, row-major) first.  Pairs of a round are disjoint (round-robin
// order); each of up to 16 pairs is taken by a group of 16 lanes.
// sig (n, decreasing).  Requires n <= 32.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(DTPB) dense_zsvals_kernel(const cplx* __restrict__ Z, int n,
                                                            int p, cplx* __restrict__ work,
                                                            double* __restrict__ sig) {
  __shared__ int nrot;
  __shared__ double nv[32];
  for (int t = threadIdx.x; t < n * p; t += blockDim.x) {
    const int a = t % n, i = t / n;
    work[(size_t)a * p + i] = Z[t];
  }
  __syncthreads();
  const int mm = n + (n & 1);
  const int half = mm / 2;
  const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (threadIdx.x == 0) nrot = 0;
    __syncthreads();
    for (int round = 0; round < mm - 1; ++round) {
      if (grp < half) {
        int a, b;
        if (grp == 0) {
          a = mm - 1;
          b = round;
        } else {
          a = (round + grp) % (mm - 1);
          b = (round - grp + (mm - 1)) % (mm - 1);
        }
        const int r0 = a < b ? a : b, r1 = a < b ? b : a;
        if (r1 < n) {
          cplx* x = work + (size_t)r0 * p;
          cplx* y = work + (size_t)r1 * p;
          double al = 0.0, be = 0.0;
          cplx ga = mk(0.0, 0.0);  // sum x conj(y)
          for (int i = gl; i < p; i += 16) {
            al += cabs2(x[i]);
            be += cabs2(y[i]);
            cfmac(ga, y[i], x[i]);
          }
          for (int o = 8; o > 0; o >>= 1) {
            al += __shfl_xor(al, o, 16);
            be += __shfl_xor(be, o, 16);
            ga.re += __shfl_xor(ga.re, o, 16);
            ga.im += __shfl_xor(ga.im, o, 16);
          }
          const double gab = sqrt(cabs2(ga));
          if (gab > 1e-300 && gab > 1e-15 * sqrt(al * be)) {
            if (gl == 0) atomicAdd(&nrot, 1);
            const double zeta = (be - al) / (2.0 * gab);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
            const cplx e = mk(ga.re / gab, ga.im / gab);  // gamma / |gamma|
            for (int i = gl; i < p; i += 16) {
              const cplx xv = x[i], ye = cmul(y[i], e);
              x[i] = csub(cscale(xv, cs), cscale(ye, sn));
              y[i] = cadd(cscale(xv, sn), cscale(ye, cs));
            }
          }
        }
      }
      __syncthreads();
    }
    if (nrot == 0) break;
    __syncthreads();
  }
  for (int a = threadIdx.x >> 6; a < n; a += blockDim.x >> 6) {
    double acc = 0.0;
    for (int i = threadIdx.x & 63; i < p; i += 64) acc += cabs2(work[(size_t)a * p + i]);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) nv[a] = sqrt(acc);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int a = 0; a < n; ++a) {
      int b = a;
      for (int c = a + 1; c < n; ++c)
        if (nv[c] > nv[b]) b = c;
      const double t = nv[a];
      nv[a] = nv[b];
      nv[b] = t;
      sig[a] = nv[a];
    }
  }
}

// Row-combination matrices that project the k columns Y out of the basis:
// Y - U~ C with C = U~^* Y (n x k):  Ik = I (k x k), Cn = -C.
__global__ void proj_mats_kernel(const cplx* __restrict__ C, int n, int k, cplx* __restrict__ Ik,
                                 cplx* __restrict__ Cn) {
  for (int t = threadIdx.x; t < k * k; t += blockDim.x)
    Ik[t] = (t % k == t / k) ? mk(1.0, 0.0) : mk(0.0, 0.0);
  for (int t = threadIdx.x; t < n * k; t += blockDim.x) Cn[t] = cscale(C[t], -1.0);
}

void launch_dense_rank_cert(hipStream_t s, const cplx* Z, int n, int p, double c, int* word) {
  const size_t sh = (n * p <= 4096) ? (size_t)n * p * sizeof(cplx) : 0;
  ALLOW_BIG_LDS(dense_rank_cert_kernel);
  hipLaunchKernelGGL(dense_rank_cert_kernel, dim3(1), dim3(DTPB), sh, s, Z, n, p, c, word);
}
void launch_dense_zsvals(hipStream_t s, const cplx* Z, int n, int p, cplx* work, double* sig) {
  hipLaunchKernelGGL(dense_zsvals_kernel, dim3(1), dim3(DTPB), 0, s, Z, n, p, work, sig);
}
void launch_proj_mats(hipStream_t s, const cplx* C, int n, int k, cplx* Ik, cplx* Cn) {
  hipLaunchKernelGGL(proj_mats_kernel, dim3(1), dim3(256), 0, s, C, n, k, Ik, Cn);
}

// ---------------------------------------------------------------------------
// Leading eigenpairs of a real symmetric matrix (n <= 64, d <= n) in one
// workgroup of four wavefronts (one per SIMD of the CU).
//  * Householder tridiagonalisation: lane r of wavefront w keeps entries
//    16w .. 16w+15 of row r in registers.  Columns k and k+1 are published
//    through LDS; each wavefront forms its part of A x (x = column k below
//    the diagonal) while the reflector's scalars are computed, so that
//    p = t A v = t (A x - alpha A e_{k+1}) needs one exchange per column.
//  * The d largest eigenvalues of T by multisection on Sturm counts, with
//    the three-term recurrence of the leading principal minors of T - x I
//    (no division; power-of-two rescaling every two terms): 256 / d lanes
//    per eigenvalue.
//  * Eigenvector j of T from a twisted factorization of T - lambda_j I (the
//    top-down and bottom-up pivots on two wavefronts at once, lane j each;
//    the twist at the smallest |gamma|); back-transform through the stored
//    reflectors and the Gram matrix of the vectors by groups of lanes, one
//    group per vector; Cholesky QR to orthonormalise in order.
// Output: lam (d, decreasing), V (n x d, column-major); bit 32 of flags[0]
// is set if the vectors are rank deficient.
// ---------------------------------------------------------------------------
namespace {
constexpr int TE_M = 64;   // largest order
constexpr int TE_LX = TE_M + 1;   // padded stride of the vector array

// 1/x to full double precision for finite x with |x| >= 1e-290: the hardware
// estimate refined by two Newton steps
__device__ __forceinline__ double te_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// square root of a positive normal x to about full precision: the hardware
// reciprocal square root estimate refined by Goldschmidt steps
__device__ __forceinline__ double te_sqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double e = fma(-g, h, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

// value of v in lane `lane` (uniform), as a scalar
__device__ __forceinline__ double te_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __hiloint2double(hi, lo);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double te_dpp(double v) {
  return dpp64<CTRL, ROWS>(v);
}

// orders LDS accesses of one wavefront around an exchange between its lanes
// (the wavefront executes them in program order; the fences keep the
// compiler from moving them across)
__device__ __forceinline__ void te_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sum over the 64 lanes of a wavefront, returned in every lane: row shifts
// accumulate each row of 16 into its last lane, the row broadcasts carry
// rows 0..2 into lane 63
__device__ __forceinline__ double te_wave_sum(double v) {
  v += te_dpp<0x111, 0xf>(v);   // row_shr:1
  v += te_dpp<0x112, 0xf>(v);   // row_shr:2
  v += te_dpp<0x114, 0xf>(v);   // row_shr:4
  v += te_dpp<0x118, 0xf>(v);   // row_shr:8
  v += te_dpp<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += te_dpp<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return te_lane(v, 63);
}

// two wavefront sums at once (independent chains, interleaved)
__device__ __forceinline__ void te_wave_sum2(double& u, double& v) {
  u += te_dpp<0x111, 0xf>(u);
  v += te_dpp<0x111, 0xf>(v);
  u += te_dpp<0x112, 0xf>(u);
  v += te_dpp<0x112, 0xf>(v);
  u += te_dpp<0x114, 0xf>(u);
  v += te_dpp<0x114, 0xf>(v);
  u += te_dpp<0x118, 0xf>(u);
  v += te_dpp<0x118, 0xf>(v);
  u += te_dpp<0x142, 0xa>(u);
  v += te_dpp<0x142, 0xa>(v);
  u += te_dpp<0x143, 0xc>(u);
  v += te_dpp<0x143, 0xc>(v);
  u = te_lane(u, 63);
  v = te_lane(v, 63);
}

template <int LEVEL>
__device__ __forceinline__ double te_bfly(double v) {
  return bfly64<LEVEL>(v);
}

// sum over aligned groups of L lanes (L a power of two, 4 <= L <= 64),
// returned in every lane of the group (the same bits in all of them)
template <int L>
__device__ __forceinline__ double te_grp_sum(double v) {
  v += te_bfly<0>(v);
  v += te_bfly<1>(v);
  if (L >= 8) v += te_bfly<2>(v);
  if (L >= 16) v += te_bfly<3>(v);
  if (L >= 32) v += __shfl_xor(v, 16, 64);
  if (L >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// max and min over aligned groups of L lanes (L a power of two <= 64)
template <int L>
__device__ __forceinline__ void te_grp_maxmin(double& mx, double& mn) {
  if (L >= 2) {
    mx = fmax(mx, te_bfly<0>(mx));
    mn = fmin(mn, te_bfly<0>(mn));
  }
  if (L >= 4) {
    mx = fmax(mx, te_bfly<1>(mx));
    mn = fmin(mn, te_bfly<1>(mn));
  }
  if (L >= 8) {
    mx = fmax(mx, te_bfly<2>(mx));
    mn = fmin(mn, te_bfly<2>(mn));
  }
  if (L >= 16) {
    mx = fmax(mx, te_bfly<3>(mx));
    mn = fmin(mn, te_bfly<3>(mn));
  }
  if (L >= 32) {
    mx = fmax(mx, __shfl_xor(mx, 16, 64));
    mn = fmin(mn, __shfl_xor(mn, 16, 64));
  }
  if (L >= 64) {
    mx = fmax(mx, __shfl_xor(mx, 32, 64));
    mn = fmin(mn, __shfl_xor(mn, 32, 64));
  }
}

// Back-transform x <- H_0 H_1 ... H_{n-3} x of the d vectors in Xv
// (Xv[c * TE_LX + i]: entry i of vector c), then the upper triangle of their
// Gram matrix into Rc (Rc[a * TE_LX + b], a <= b).  Group c of L lanes owns
// vector c, lane s of the group its entries s, s + L, ...
template <int L>
__device__ void te_back_gram(const double* __restrict__ H, const double* __restrict__ tau,
                             double* __restrict__ Xv, double* __restrict__ Rc,
                             const double* __restrict__ znrm, int n, int d) {
  constexpr int R = TE_M / L;
  const int c = threadIdx.x / L, sub = threadIdx.x & (L - 1);
  const bool act = c < d;
  const int cc = act ? c : 0;
  // unit vectors (the scale of each is irrelevant to the orthonormalisation
  // that follows, but keeps the Gram entries in range)
  const double inv = 1.0 / sqrt(znrm[cc] + znrm[TE_M + cc]);
  double x[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int i = sub + L * t;
    const double v = Xv[cc * TE_LX + i];
    x[t] = (act && i < n) ? v * inv : 0.0;
  }
  // reflector k and its scalar, loaded one step ahead
  double h[R];
  double tk = 0.0;
  if (n >= 3) {
    tk = tau[n - 3];
#pragma unroll
    for (int t = 0; t < R; ++t) h[t] = H[(n - 3) * TE_M + sub + L * t];
  }
  for (int k = n - 3; k >= 0; --k) {
    const int kn = max(k - 1, 0);
    const double tkn = tau[kn];
    double hn[R];
#pragma unroll
    for (int t = 0; t < R; ++t) hn[t] = H[kn * TE_M + sub + L * t];
    if (tk != 0.0) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        if (t & 1)
          s1 = fma(h[t], x[t], s1);
        else
          s0 = fma(h[t], x[t], s0);
      }
      const double sc = tk * te_grp_sum<L>(s0 + s1);
#pragma unroll
      for (int t = 0; t < R; ++t) x[t] = fma(-sc, h[t], x[t]);
    }
    tk = tkn;
#pragma unroll
    for (int t = 0; t < R; ++t) h[t] = hn[t];
  }
  __syncthreads();   // every group has read its input
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int i = sub + L * t;
    if (act && i < n) Xv[c * TE_LX + i] = x[t];
  }
  __syncthreads();
  // row c of the Gram matrix: all groups read vector j at the same time
  for (int j = 0; j < d; ++j) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = sub + L * t;
      const double xv = Xv[j * TE_LX + i];
      const double xj = (i < n) ? xv : 0.0;
      if (t & 1)
        s1 = fma(x[t], xj, s1);
      else
        s0 = fma(x[t], xj, s0);
    }
    const double g = te_grp_sum<L>(s0 + s1);
    if (act && sub == 0 && j >= c) Rc[c * TE_LX + j] = g;
  }
}
}  // namespace

__global__ void __launch_bounds__(256) dense_topeig_kernel(const double* __restrict__ G, int n, int d,
                                                           double* __restrict__ V,
                                                           double* __restrict__ lam,
                                                           double* __restrict__ Mc,
                                                           int* __restrict__ flags,
                                                           const int* __restrict__ stop) {
  if (stop && *stop) return;
  constexpr int M = TE_M;
  constexpr int CW = 16;                // columns per wavefront
  __shared__ double H[M * M];          // H[k * M + i]: reflector k (zero for i <= k)
  __shared__ double W[3 * M * M];      // Sturm data; elimination factors; vectors and Gram
  __shared__ double colk[M], colk1[M]; // columns k and k + 1
  __shared__ double ps[4 * M];         // per-wavefront parts of A x
  __shared__ double dcor[M];           // corrections of the diagonal
  __shared__ double wbuf[4 * M];       // per-wavefront copies of w
  __shared__ double qsw[8];            // per-wavefront parts of x^T A x and |x|^2
  __shared__ double tau[M], dd[M], ee[M], lamg[M];
  __shared__ double red[8];
  __shared__ int badf;
  const int tid = threadIdx.x, r = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
#ifdef SYMROM_TOPEIG_TIMING
  unsigned long long tsv[6];
  tsv[0] = wall_clock64();
#define TS(k) tsv[k] = wall_clock64()
  unsigned long long tiv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#define TIV(k) tiv[k] = wall_clock64()
  long long seg[5] = {0, 0, 0, 0, 0};
  long long tprev = clock64();
#define SEG(i)                  \
  {                             \
    long long tn = clock64();   \
    seg[i] += tn - tprev;       \
    tprev = tn;                 \
  }
#else
#define TS(k)
#define TIV(k)
#define SEG(i)
#endif
  // ---- tridiagonalisation ----
  // The matrix is first scaled by a power of two (exact) so that its largest
  // entry lies in [1/2, 1): the reflector scalars then stay far from under-
  // and overflow.  The eigenvalues are scaled back at the end.
  double a[CW];
  double gmx = 0.0;
#pragma unroll
  for (int jj = 0; jj < CW; ++jj) {
    const int j = CW * w + jj;
    a[jj] = (r < n && j < n) ? G[(size_t)j * n + r] : 0.0;
    gmx = fmax(gmx, fabs(a[jj]));
  }
  for (int o = 32; o > 0; o >>= 1) gmx = fmax(gmx, __shfl_xor(gmx, o, 64));
  if (r == 0) red[w] = gmx;
  __syncthreads();
  gmx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const int gex = (gmx > 0.0) ? __builtin_amdgcn_frexp_exp(gmx) : 0;
#pragma unroll
  for (int jj = 0; jj < CW; ++jj) a[jj] = __builtin_amdgcn_ldexp(a[jj], -gex);
  double* wb = wbuf + w * M;
  for (int k = 0; k + 2 < n; ++k) {
    // Rows k and k+1 (the trailing matrix is symmetric: they are columns k
    // and k+1) are published by lanes k and k+1 of every wavefront, each for
    // its own 16 columns; then the processed part of row k (columns <= k) is
    // cleared by the lanes of the same wavefront (stores of one wavefront to
    // LDS take effect in program order).
    if (r == k || r == k + 1) {
      double* dst = (r == k ? colk : colk1) + CW * w;
#pragma unroll
      for (int jj = 0; jj < CW; jj += 2)
        *reinterpret_cast<double2*>(dst + jj) = make_double2(a[jj], a[jj + 1]);
    }
    if (r >= CW * w && r < CW * w + CW && r <= k) colk[r] = 0.0;
    SEG(0);
    __syncthreads();
    SEG(1);
    // x (row k right of the diagonal), this wavefront's part of A x and of
    // x^T A x, |x|^2, and the reflector I - t v v^T with v = x - alpha e_{k+1}
    const double xr = colk[r];          // zero for r <= k
    const double a1 = colk1[r];         // A[r][k+1]
    const double x0 = colk[k + 1];
    const double a11 = colk1[k + 1];
    double xj[CW];
#pragma unroll
    for (int jj = 0; jj < CW; jj += 2) {
      const double2 q = *reinterpret_cast<const double2*>(colk + CW * w + jj);
      xj[jj] = q.x;
      xj[jj + 1] = q.y;
    }
    double pw = 0.0, pw2 = 0.0;
#pragma unroll
    for (int jj = 0; jj < CW; jj += 2) {
      pw = fma(a[jj], xj[jj], pw);
      pw2 = fma(a[jj + 1], xj[jj + 1], pw2);
    }
    pw += pw2;
    ps[w * M + r] = pw;
    double qw = xr * pw, sig = xr * xr;
    te_wave_sum2(qw, sig);
    if (r == 0) qsw[w] = qw;
    double t = 0.0, alpha = x0;
    if (sig > 1e-280) {
      const double sq = te_sqrt(sig);
      const double al = (x0 >= 0.0) ? -sq : sq;
      const double vn2 = 2.0 * sig - 2.0 * al * x0;
      if (vn2 > 1e-280) {
        t = 2.0 * te_rcp(vn2);
        alpha = al;
      }
    }
    const double vr = (r > k && r < n) ? (r == k + 1 ? xr - alpha : xr) : 0.0;
    if (w == 0) {
      H[k * M + r] = vr;
      if (r == 0) {
        tau[k] = t;
        ee[k] = alpha;
      }
    }
    SEG(2);
    __syncthreads();
    SEG(3);
    if (t != 0.0) {
      // p = t A v = t (A x - alpha A e_{k+1});  v^T p = t (x^T A x -
      // 2 alpha (A x)_{k+1} + alpha^2 A_{k+1,k+1});  w = p - (t/2)(v^T p) v
      const double ax = ((ps[r] + ps[M + r]) + ps[2 * M + r]) + ps[3 * M + r];
      const double ax1 =
          ((ps[k + 1] + ps[M + k + 1]) + ps[2 * M + k + 1]) + ps[3 * M + k + 1];
      const double xax = ((qsw[0] + qsw[1]) + qsw[2]) + qsw[3];
      const double pr = (r > k && r < n) ? t * (ax - alpha * a1) : 0.0;
      const double kv = t * ((xax - 2.0 * alpha * ax1) + alpha * alpha * a11);
      const double wr = pr - 0.5 * t * kv * vr;   // zero for r <= k
      // A <- A - v w^T - w v^T, with x in place of v for the column factor:
      // the difference, alpha w in column k+1, is never read again except
      // on the diagonal, which is corrected at the end
      if (w == 0 && r == k + 1) dcor[r] = alpha * wr;
      wb[r] = wr;
      double wj[CW];
#pragma unroll
      for (int jj = 0; jj < CW; jj += 2) {
        const double2 q = *reinterpret_cast<const double2*>(wb + CW * w + jj);
        wj[jj] = q.x;
        wj[jj + 1] = q.y;
      }
#pragma unroll
      for (int jj = 0; jj < CW; ++jj) a[jj] = fma(-vr, wj[jj], fma(-wr, xj[jj], a[jj]));
    } else if (w == 0 && r == k + 1) {
      dcor[r] = 0.0;
    }
    SEG(4);
  }
  __syncthreads();
  {
    // diagonal and last subdiagonal entry from the wavefront owning the column
    // (column k+1 of step k holds A - v w^T - w x^T: its diagonal entry
    // misses alpha w_{k+1}, and the last subdiagonal entry is read from row
    // n-2, whose column n-1 was never such a column)
#pragma unroll
    for (int jj = 0; jj < CW; ++jj) {
      const int j = CW * w + jj;
      if (j == r && r < n) dd[r] = a[jj] + ((r >= 1 && r + 1 < n) ? dcor[r] : 0.0);
      if (n >= 2 && j == n - 1 && r == n - 2) ee[n - 2] = a[jj];
    }
    if (w == 0 && (r == n - 1 || r >= n)) ee[r] = 0.0;
    __syncthreads();
  }
  TS(1);
  // ---- d largest eigenvalues by multisection ----
  // Gershgorin interval, in wavefront 0 (lane i: row i)
  if (w == 0) {
    const double ddr = dd[r], eer = ee[r], eem = ee[r > 0 ? r - 1 : 0];
    const double di = (r < n) ? ddr : 0.0;
    const double rad = (r < n) ? fabs(r > 0 ? eem : 0.0) + fabs(eer) : 0.0;
    double lo = (r < n) ? di - rad : INFINITY, hi = (r < n) ? di + rad : -INFINITY;
    for (int o = 32; o > 0; o >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, o, 64));
      hi = fmax(hi, __shfl_xor(hi, o, 64));
    }
    if (r == 0) {
      red[0] = lo;
      red[1] = hi;
    }
  }
  __syncthreads();
  const double lo = red[0], hi = red[1];
  // power-of-two scale: T / sc exactly, entries of modulus <= 1
  const double amax = fmax(fabs(lo), fabs(hi));
  const double sc = (amax > 0.0) ? __builtin_amdgcn_ldexp(1.0, __builtin_amdgcn_frexp_exp(amax)) : 1.0;
  const double isc = 1.0 / sc;
  // (d_i, e_{i-1}^2) of T / sc, one LDS read per term; eight padding terms
  // with d = 4 (above every shift) leave the count unchanged
  double2* de = reinterpret_cast<double2*>(W);
  if (tid < n + 8) {
    const double ep = (tid > 0 && tid < n) ? ee[tid - 1] * isc : 0.0;
    de[tid] = (tid < n) ? make_double2(dd[tid] * isc, ep * ep) : make_double2(4.0, 0.0);
  }
  // every pivot (ratio of consecutive minors) is moved away from zero by
  // pivmin in its own direction: no effect above 1e-44 of the pivot, and no
  // zero minor (a perturbation of T / sc far below rounding)
  const double pivmin = 1e-60;
  // ms lanes per eigenvalue (a power of two, so a group never straddles a
  // wavefront and its bracket update is a butterfly over ms lanes)
  int ms = 1;
  while (ms * 2 <= 64 && ms * 2 * d <= 256) ms *= 2;
  const int grp = tid / ms, sub = tid % ms;
  const bool gact = grp < d;
  const int kk = n - 1 - (gact ? grp : 0);       // eigenvalue kk in increasing order
  __syncthreads();
  double a0 = lo * isc, b0 = hi * isc;
  const double frac = (double)(sub + 1) / (double)(ms + 1);
  for (int it = 0; it < 200; ++it) {
    const bool more = gact && (b0 - a0 > 2.2e-16);
    if (!__syncthreads_or(more)) break;
    const double x = fma(b0 - a0, frac, a0);
    // count of negative ratios P_{i+1} / P_i of the leading minors of
    // T / sc - x I (the negative pivots of its LDL^T factorisation)
    double pa = 1.0, pb = 0.0;   // P_i, P_{i-1}
    unsigned cnt = 0;
    double2 c0 = de[0], c1 = de[1], c2 = de[2], c3 = de[3];
    for (int i = 0; i < n; i += 4) {
      const double2 n0 = de[i + 4], n1 = de[i + 5], n2 = de[i + 6], n3 = de[i + 7];
#define TE_STURM(C)                                                            \
  {                                                                            \
    double pn = fma((C).x - x, pa, -(C).y * pb);                               \
    pn += copysign(pivmin * fabs(pa), pn);                                     \
    cnt += (unsigned)(__double2hiint(pn) ^ __double2hiint(pa)) >> 31;          \
    pb = pa;                                                                   \
    pa = pn;                                                                   \
  }
      TE_STURM(c0)
      TE_STURM(c1)
      TE_STURM(c2)
      TE_STURM(c3)
#undef TE_STURM
      // rescale by a power of two (exact): at most a factor 6^4 of growth and
      // pivmin^4 of decay between two rescalings
      const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(pa), fabs(pb)));
      pa = __builtin_amdgcn_ldexp(pa, -ex);
      pb = __builtin_amdgcn_ldexp(pb, -ex);
      c0 = n0;
      c1 = n1;
      c2 = n2;
      c3 = n3;
    }
    // new bracket: the largest point with count <= kk and the smallest with
    // count > kk, by a butterfly over the group (max / min: order-free)
    double na = ((int)cnt <= kk) ? x : a0;
    double nb = ((int)cnt > kk) ? x : b0;
    switch (ms) {
      case 64: te_grp_maxmin<64>(na, nb); break;
      case 32: te_grp_maxmin<32>(na, nb); break;
      case 16: te_grp_maxmin<16>(na, nb); break;
      case 8: te_grp_maxmin<8>(na, nb); break;
      case 4: te_grp_maxmin<4>(na, nb); break;
      case 2: te_grp_maxmin<2>(na, nb); break;
      default: break;
    }
    if (more) {
      if (!(na > a0) && !(nb < b0)) {
        b0 = a0;   // no interior point is representable: converged
      } else {
        a0 = na;
        b0 = nb;
      }
    }
  }
  if (gact && sub == 0) lamg[grp] = 0.5 * (a0 + b0) * sc;
  __syncthreads();
  TS(2);
  // ---- eigenvectors of T by twisted factorizations of T/sc - lambda I ----
  // For lane c < d (eigenvalue lambda_c): wavefront 0 forms the top-down
  // LDL^T pivots delta_i, wavefront 1 at the same time the bottom-up pivots
  // rho_i and multipliers u_i = e_i / rho_{i+1}; the twist index k minimises
  // |gamma_i|, gamma_i = delta_i + rho_i - (d_i - lambda); then z_k = 1,
  // z_i = -(e_i / delta_i) z_{i+1} above k (wavefront 0) and
  // z_{i+1} = -u_i z_i below k (wavefront 1).  Pivots are kept at least
  // ptiny in modulus (a perturbation of T / sc of that size).
  const double ptiny = 2.2e-16;
  double* Dlt = W;                  // delta_i: Dlt[i * M + c]
  double* Uup = W + M * M;          // u_i
  double* Rho = W + 2 * M * M;      // rho_i
  double* Xv = W + 2 * M * M - M;   // vectors, Xv[c * TE_LX + i] (after the pivots; the
                                    // rows it covers of Uup (i = 63) and Rho are unused then)
  double* Rc = W;                   // Gram matrix, then Cholesky factor
  __shared__ double2 dsc[M + 4];    // (d_i, e_i) of T / sc
  __shared__ double znrm[2 * M];    // squared norms of the two halves of each z
  if (tid < M + 4)
    dsc[tid] = (tid < n) ? make_double2(dd[tid] * isc, ee[tid] * isc) : make_double2(0.0, 0.0);
  __syncthreads();
  const double lv = lamg[min(r, max(d - 1, 0))] * isc;
  auto guard = [&](double v) { return copysign(fmax(fabs(v), ptiny), v); };
  if (w == 0 && d > 0) {
    double dl = guard(dsc[0].x - lv);
    Dlt[r] = dl;
    double2 dA = dsc[1], dB = dsc[2];
    for (int i = 0; i + 1 < n; ++i) {
      const double2 dn = dA;
      const double2 dC = dsc[i + 3];
      dA = dB;
      dB = dC;
      const double e = dsc[i].y;
      const double l = e * te_rcp(dl);
      dl = guard(fma(-l, e, dn.x - lv));
      Dlt[(i + 1) * M + r] = dl;
    }
  } else if (w == 1 && d > 0) {
    double rh = guard(dsc[n - 1].x - lv);
    Rho[(n - 1) * M + r] = rh;
    for (int i = n - 2; i >= 0; --i) {
      const double2 di = dsc[i];
      const double u = di.y * te_rcp(rh);
      Uup[i * M + r] = u;
      rh = guard(fma(-u, di.y, di.x - lv));
      Rho[i * M + r] = rh;
    }
  }
  __syncthreads();
  // twist index (both wavefronts, the same in each lane)
  int k = 0;
  if (w < 2 && d > 0) {
    double best = INFINITY;
    for (int i = 0; i < n; ++i) {
      const double g = fabs(Dlt[i * M + r] + Rho[i * M + r] - (dsc[i].x - lv));
      if (g < best) {
        best = g;
        k = i;
      }
    }
  }
  __syncthreads();   // (the vectors overwrite the rho_i)
  if (w < 2 && d > 0) {
    double z = 1.0, nz = 0.0;
    if (w == 0) {
      // z_k and the entries above it
      Xv[r * TE_LX + k] = 1.0;
      nz = 1.0;
      for (int i = n - 2; i >= 0; --i) {
        const double l = dsc[i].y * te_rcp(Dlt[i * M + r]);
        if (i < k) {
          z = -l * z;
          Xv[r * TE_LX + i] = z;
          nz = fma(z, z, nz);
        }
      }
    } else {
      // the entries below z_k
      for (int i = 0; i + 1 < n; ++i) {
        const double u = Uup[i * M + r];
        if (i >= k) {
          z = -u * z;
          Xv[r * TE_LX + i + 1] = z;
          nz = fma(z, z, nz);
        }
      }
    }
    znrm[w * M + r] = nz;
  }
  __syncthreads();
  TS(3);
  // ---- back-transform and Gram matrix, one group of lanes per vector ----
  {
    int L = 64;
    while (L > 4 && L * d > 256) L >>= 1;
    switch (L) {
      case 64: te_back_gram<64>(H, tau, Xv, Rc, znrm, n, d); break;
      case 32: te_back_gram<32>(H, tau, Xv, Rc, znrm, n, d); break;
      case 16: te_back_gram<16>(H, tau, Xv, Rc, znrm, n, d); break;
      case 8: te_back_gram<8>(H, tau, Xv, Rc, znrm, n, d); break;
      default: te_back_gram<4>(H, tau, Xv, Rc, znrm, n, d); break;
    }
  }
  __syncthreads();
  TS(4);
  // ---- Cholesky factor R of the Gram matrix (right-looking, wavefront 0;
  //      lane b owns column b), then V = X R^{-1} ----
  if (w == 0) {
    int bad = 0;
    for (int j = 0; j < d; ++j) {
      const double gjj = Rc[j * TE_LX + j];
      if (!(gjj > 0.0)) {
        bad = 1;
        break;
      }
      const double rjj = sqrt(gjj);
      const double ri = 1.0 / rjj;
      double rjb = 0.0;
      if (r > j && r < d) {
        rjb = Rc[j * TE_LX + r] * ri;
        Rc[j * TE_LX + r] = rjb;
      }
      if (r == j) Rc[j * TE_LX + j] = rjj;
      te_wave_sync();
      if (r > j && r < d)
        for (int q = j + 1; q <= r; ++q) Rc[q * TE_LX + r] -= Rc[j * TE_LX + q] * rjb;
      te_wave_sync();
    }
    if (r == 0) badf = bad;
  }
  __syncthreads();
  const int bad = badf;
  if (!bad && tid < n) {
    // row tid of X R^{-1} by forward substitution, in place
    for (int c = 0; c < d; ++c) {
      double s = Xv[c * TE_LX + tid];
      for (int q = 0; q < c; ++q) s = fma(-Xv[q * TE_LX + tid], Rc[q * TE_LX + c], s);
      s /= Rc[c * TE_LX + c];
      Xv[c * TE_LX + tid] = s;
      V[(size_t)c * n + tid] = s;
      if (Mc) {
        // the DEIM basis coefficients V[:, c] / sqrt(lambda_c)
        const double l = __builtin_amdgcn_ldexp(lamg[c], gex);
        Mc[(size_t)c * n + tid] = (l > 0.0) ? s / sqrt(l) : 0.0;
      }
    }
  }
  if (tid < d) {
    const double l = __builtin_amdgcn_ldexp(lamg[tid], gex);
    lam[tid] = l;
    if (Mc && !(l > 0.0) && flags) atomicOr(&flags[0], 8);
  }
  if (tid == 0 && bad && flags) atomicOr(&flags[0], 32);
#ifdef SYMROM_TOPEIG_TIMING
  TS(5);
  if (tid == 0 && flags)
    for (int k = 0; k < 6; ++k) flags[8 + k] = (int)(tsv[k] - tsv[0]);
  if ((tid & 63) == 0 && flags)
    for (int k = 0; k < 5; ++k) flags[16 + 8 * w + k] = (int)seg[k];
  if (tid == 0 && flags)
    for (int k = 1; k < 7; ++k) flags[48 + k] = (int)(tiv[k] - tiv[0]);
#endif
#undef TS
#undef TIV
#undef SEG
}

void launch_dense_topeig(hipStream_t s, const double* G, int n, int d, double* V, double* lam,
                         int* flags, const int* stop, double* Mc) {
  hipLaunchKernelGGL(dense_topeig_kernel, dim3(1), dim3(256), 0, s, G, n, d, V, lam, Mc, flags,
                     stop);
}
