// Streaming kernels of the reduced model: field gather at reconstructed
// particles, tall-skinny products with reduction over particles (split over
// row blocks, reduced in a fixed order), and row-wise small products.
#include "common.h"
#include "kernels.h"

// ---------------------------------------------------------------------------
// Gather (eq. grH-full): for every particle row l and parameter i, rebuild
// x = Re(U~[l,:] Z~[:,i]) and v = Im(U~[l,:] Z~[:,i]), look the field of the
// cell up, F = (q/m) e_i[j(x)], and write
//   FULL = false:  F (real, N x p)               -- position gradient only
//   FULL = true :  G~ = F + i v (complex, N x p)  -- [G_X; G_V] in complex form
// The basis row lives in registers, the coefficient tile and the field table
// of the block's parameter tile in LDS.
// ---------------------------------------------------------------------------
template <int NC, bool FULL>
__global__ void __launch_bounds__(512) gather_rom_kernel(
    const cplx* __restrict__ U, int N, int n, const cplx* __restrict__ Z, int p, int Nx, int pt,
    int rpb, const double* __restrict__ factor, const double* __restrict__ e, double qm,
    const int* __restrict__ active, void* __restrict__ out) {
  extern __shared__ double smem[];
  double* et = smem;                                   // pt * Nx
  cplx* Zs = reinterpret_cast<cplx*>(smem + pt * Nx);  // pt * NC
  const int p0 = blockIdx.y * pt;
  const int np = min(pt, p - p0);
  for (int t = threadIdx.x; t < np * Nx; t += blockDim.x) et[t] = qm * e[(size_t)p0 * Nx + t];
  for (int t = threadIdx.x; t < np * NC; t += blockDim.x) {
    int i = t / NC, k = t % NC;
    Zs[t] = (k < n) ? Z[(size_t)(p0 + i) * n + k] : mk(0.0, 0.0);
  }
  __syncthreads();
  const int r0 = blockIdx.x * rpb;
  const int r1 = min(N, r0 + rpb);
  for (int l = r0 + threadIdx.x; l < r1; l += blockDim.x) {
    cplx u[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) u[k] = (k < n) ? U[(size_t)k * N + l] : mk(0.0, 0.0);
    for (int i = 0; i < np; ++i) {
      if (active && !active[p0 + i]) continue;
      const cplx* zi = Zs + i * NC;
      double x0 = 0.0, x1 = 0.0, v0 = 0.0, v1 = 0.0;
#pragma unroll
      for (int k = 0; k < NC; k += 2) {
        x0 = fma(u[k].re, zi[k].re, x0);
        x0 = fma(-u[k].im, zi[k].im, x0);
        x1 = fma(u[k + 1].re, zi[k + 1].re, x1);
        x1 = fma(-u[k + 1].im, zi[k + 1].im, x1);
        if (FULL) {
          v0 = fma(u[k].re, zi[k].im, v0);
          v0 = fma(u[k].im, zi[k].re, v0);
          v1 = fma(u[k + 1].re, zi[k + 1].im, v1);
          v1 = fma(u[k + 1].im, zi[k + 1].re, v1);
        }
      }
      const double x = x0 + x1;
      int j;
      double th;
      cell_of(x, factor[p0 + i], Nx, j, th);
      const double F = et[i * Nx + j];
      const size_t o = (size_t)(p0 + i) * N + l;
      if (FULL)
        reinterpret_cast<cplx*>(out)[o] = mk(F, v0 + v1);
      else
        reinterpret_cast<double*>(out)[o] = F;
    }
  }
}

// Reconstruct X = Re(U~ Z~), V = Im(U~ Z~) (N x p each).
template <int NC>
__global__ void __launch_bounds__(256) reconstruct_kernel(const cplx* __restrict__ U, int N, int n,
                                                          const cplx* __restrict__ Z, int p,
                                                          double* __restrict__ X,
                                                          double* __restrict__ V) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= N) return;
  cplx u[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) u[k] = (k < n) ? U[(size_t)k * N + l] : mk(0.0, 0.0);
  for (int i = 0; i < p; ++i) {
    cplx acc = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < NC; ++k)
      if (k < n) cfma(acc, u[k], Z[(size_t)i * n + k]);
    if (X) X[(size_t)i * N + l] = acc.re;
    if (V) V[(size_t)i * N + l] = acc.im;
  }
}

// ---------------------------------------------------------------------------
// Split-K product C = A^* B with A = [A_0 ... ] (N x a, complex) and
// B = [B_0 ... ] (N x b, complex, or real when b_real).  Block kb reduces the
// rows [kb*rk, (kb+1)*rk) in tiles of TR rows staged through LDS and writes
// its a x b partial; reduce_partials_kernel sums the blocks in order.
// ---------------------------------------------------------------------------
#define GEMM_TR 32

__device__ inline const cplx* list_col(const MatList& L, int c, int& local) {
  int s = 0;
  while (s < L.count - 1 && c >= L.cols[s]) {
    c -= L.cols[s];
    ++s;
  }
  local = c;
  return L.ptr[s];
}

// Each thread owns a 4 x 4 tile of C (4 columns of A, 4 columns of B) and a
// row group: the R = 256 / tiles threads of a tile take every R-th row of
// the block's range.  Rows arrive in chunks of TR staged through LDS with
// coalesced loads (each element read from memory once per block; one copy
// when A and B are the same list), and the R partial tiles are summed in
// LDS in a fixed order.  Requires a, b <= 64.
// ---------------------------------------------------------------------------
#define GEMM_RED_LD 257
__global__ void __launch_bounds__(256) gemm_ah_b_kernel(MatList A, int a, MatList B, int b,
                                                        int flags, int N, int rk, int TR,
                                                        cplx* __restrict__ part) {
  extern __shared__ cplx sm[];   // staging [a (+ b)][TR], later the tile sums [16][GEMM_RED_LD]
  __shared__ const void* colp[128];
  const bool b_real = flags & GEMM_B_REAL;
  const bool a_real = flags & GEMM_A_REAL;
  const bool conj_a = !(flags & GEMM_NO_CONJ_A);
  const bool same = flags & GEMM_SAME;
  const int tid = threadIdx.x;
  const int nst = same ? a : a + b;   // staged columns
  if (tid < nst) {
    const bool isA = tid < a;
    int lc;
    const cplx* base = isA ? list_col(A, tid, lc) : list_col(B, tid - a, lc);
    const bool re = isA ? a_real : b_real;
    colp[tid] = re ? static_cast<const void*>(reinterpret_cast<const double*>(base) + (size_t)lc * N)
                   : static_cast<const void*>(base + (size_t)lc * N);
  }
  const int kb = blockIdx.x;
  const int r0 = kb * rk;
  const int r1 = min(N, r0 + rk);
  const int nta = (a + 3) / 4;
  const int ntb = (b + 3) / 4;
  const int nt = nta * ntb;
  const int R = max(1, 256 / nt);
  const int tile = tid / R;
  const int rg = tid % R;
  const bool owner = tile < nt;
  const int ta0 = (tile % nta) * 4;
  const int tb0 = (tile / nta) * 4;
  cplx* sA = sm;
  cplx* sB = same ? sm : sm + (size_t)a * TR;
  cplx acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = mk(0.0, 0.0);
  for (int c0 = r0; c0 < r1; c0 += TR) {
    const int tn = min(TR, r1 - c0);
    __syncthreads();
    // stage the chunk: element t = col * TR + row; up to 16 loads in flight
    const int tot = nst * TR;
    for (int t0 = 0; t0 < tot; t0 += 16 * 256) {
      cplx v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int t = t0 + u * 256 + tid;
        v[u] = mk(0.0, 0.0);
        if (t < tot) {
          const int col = t / TR, row = t % TR;
          if (row < tn) {
            const bool re = (col < a) ? a_real : b_real;
            v[u] = re ? mk(reinterpret_cast<const double*>(colp[col])[c0 + row], 0.0)
                      : reinterpret_cast<const cplx*>(colp[col])[c0 + row];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int t = t0 + u * 256 + tid;
        if (t < tot) sm[t] = v[u];
      }
    }
    __syncthreads();
    if (owner) {
      for (int row = rg; row < tn; row += R) {
        cplx av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const cplx x = (ta0 + i < a) ? sA[(ta0 + i) * TR + row] : mk(0.0, 0.0);
          av[i] = conj_a ? x : cconj(x);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = (tb0 + j < b) ? sB[(tb0 + j) * TR + row] : mk(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) cfmac(acc[i][j], av[i], bv[j]);
      }
    }
  }
  __syncthreads();
  // tile sums, entry-major with a padded stride (GEMM_RED_LD = 257 complex):
  // the writes of a wavefront are consecutive and the reads of different
  // entries fall in different banks
  cplx* red = sm;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[(i * 4 + j) * GEMM_RED_LD + tid] = acc[i][j];
  __syncthreads();
  // sum the R row groups of every (tile, entry) in a fixed order, one
  // output entry per thread at a time
  const int nout = a * b;
  for (int o = tid; o < nt * 16; o += blockDim.x) {
    const int tl = o / 16, q = o % 16;
    cplx sm2 = mk(0.0, 0.0);
    // in order; unrolled so that the independent LDS loads are batched
#pragma unroll 8
    for (int g = 0; g < R; ++g) sm2 = cadd(sm2, red[q * GEMM_RED_LD + tl * R + g]);
    const int ia = (tl % nta) * 4 + q / 4, ib = (tl / nta) * 4 + q % 4;
    if (ia < a && ib < b) part[(size_t)kb * nout + (size_t)ib * a + ia] = sm2;
  }
}

// C[o] = sum_k part[k][o], k in a fixed order: one wavefront per output,
// lane-strided partial sums combined by a fixed butterfly.
__global__ void __launch_bounds__(256) reduce_partials_kernel(const cplx* __restrict__ part,
                                                              int nkb, int nout,
                                                              cplx* __restrict__ C) {
  const int lane = threadIdx.x & 63;
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (o >= nout) return;
  double re = 0.0, im = 0.0;
  for (int k = lane; k < nkb; k += 64) {
    const cplx v = part[(size_t)k * nout + o];
    re += v.re;
    im += v.im;
  }
  for (int s = 32; s > 0; s >>= 1) {
    re += __shfl_xor(re, s, 64);
    im += __shfl_xor(im, s, 64);
  }
  if (lane == 0) C[o] = mk(re, im);
}

// ---------------------------------------------------------------------------
// Row-wise combination out = sum_s In_s M_s with In_s (N x k_s) complex and
// M_s (k_s x m) small complex matrices (column-major, ld k_s) held in LDS.
// One thread per row; safe in place (out may alias an input).
// ---------------------------------------------------------------------------
template <int MC>
__global__ void __launch_bounds__(256) rowgemm_kernel(RowTerms T, int N, int m, cplx* out) {
  extern __shared__ cplx Ms[];
  int off = 0;
  for (int s = 0; s < T.count; ++s) {
    for (int t = threadIdx.x; t < T.k[s] * m; t += blockDim.x) Ms[off + t] = T.M[s][t];
    off += T.k[s] * m;
  }
  __syncthreads();
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= N) return;
  cplx acc[MC];
#pragma unroll
  for (int o = 0; o < MC; ++o) acc[o] = mk(0.0, 0.0);
  off = 0;
  for (int s = 0; s < T.count; ++s) {
    const cplx* in = T.in[s];
    const int ks = T.k[s];
    for (int k = 0; k < ks; ++k) {
      const cplx v = in[(size_t)k * N + l];
      const cplx* mrow = Ms + off + k;  // M[k][o] at mrow[o * ks]
#pragma unroll
      for (int o = 0; o < MC; ++o)
        if (o < m) cfma(acc[o], v, mrow[o * ks]);
    }
    off += ks * m;
  }
#pragma unroll
  for (int o = 0; o < MC; ++o)
    if (o < m) out[(size_t)o * N + l] = acc[o];
}

// ---------------------------------------------------------------------------
// DEIM gather (eq. grHDD with the exact potential): for the d sampled rows
// I_r, g_F[k,i] = sum_r conj(U~[I_r,k]) w_r (q/m) e_i[j(x_{I_r,i})].
// One block per parameter; threads over k.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) deim_gather_kernel(
    const cplx* __restrict__ U, int N, int n, const cplx* __restrict__ Z, int p, int Nx,
    const double* __restrict__ factor, const double* __restrict__ e, double qm,
    const int* __restrict__ idx, const double* __restrict__ w, int d,
    const int* __restrict__ active, cplx* __restrict__ gF) {
  __shared__ double Fw[256];
  const int i = blockIdx.x;
  if (active && !active[i]) return;
  const cplx* zi = Z + (size_t)i * n;
  for (int r = threadIdx.x; r < d; r += blockDim.x) {
    const int l = idx[r];
    double x = 0.0;
    for (int k = 0; k < n; ++k) {
      cplx u = U[(size_t)k * N + l];
      x = fma(u.re, zi[k].re, x);
      x = fma(-u.im, zi[k].im, x);
    }
    int j;
    double th;
    cell_of(x, factor[i], Nx, j, th);
    Fw[r] = w[r] * qm * e[(size_t)i * Nx + j];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    cplx s = mk(0.0, 0.0);
    for (int r = 0; r < d; ++r) {
      cplx u = U[(size_t)k * N + idx[r]];
      s.re = fma(u.re, Fw[r], s.re);
      s.im = fma(-u.im, Fw[r], s.im);
    }
    gF[(size_t)i * n + k] = s;
  }
}

// DEIM snapshot Lambda^0(X_r^i) Phi^i at every particle (Sec. 4.3, eq. Ydeim)
// for the parameters sub[0..psub): (1 - theta) Phi_j + theta Phi_{j+1},
// written as column c of Y (N x psub).
template <int NC>
__global__ void __launch_bounds__(256) snapshot_kernel(const cplx* __restrict__ U, int N, int n,
                                                       const cplx* __restrict__ Z,
                                                       const int* __restrict__ sub, int psub,
                                                       int Nx, const double* __restrict__ factor,
                                                       const double* __restrict__ phi,
                                                       double* __restrict__ Y) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= N) return;
  cplx u[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) u[k] = (k < n) ? U[(size_t)k * N + l] : mk(0.0, 0.0);
  for (int c = 0; c < psub; ++c) {
    const int i = sub[c];
    double x0 = 0.0, x1 = 0.0;
#pragma unroll
    for (int k = 0; k < NC; k += 2) {
      if (k < n) {
        cplx z = Z[(size_t)i * n + k];
        x0 = fma(u[k].re, z.re, x0);
        x0 = fma(-u[k].im, z.im, x0);
      }
      if (k + 1 < n) {
        cplx z = Z[(size_t)i * n + k + 1];
        x1 = fma(u[k + 1].re, z.re, x1);
        x1 = fma(-u[k + 1].im, z.im, x1);
      }
    }
    int j;
    double th;
    cell_of(x0 + x1, factor[i], Nx, j, th);
    int j1 = (j + 1 == Nx) ? 0 : j + 1;
    const double* ph = phi + (size_t)i * Nx;
    Y[(size_t)c * N + l] = (1.0 - th) * ph[j] + th * ph[j1];
  }
}

// out (N x d) = sum_s in_s (N x kin) * M[s*kin : (s+1)*kin, :] with M (P x d,
// column-major, ld ldM): the DEIM basis Psi = Y V diag(lam)^{-1/2}.
template <int MC>
__global__ void __launch_bounds__(256) rowgemm_real_kernel(RealList L, int kin, int N,
                                                           const double* __restrict__ M, int ldM,
                                                           int d, double* __restrict__ out) {
  extern __shared__ double Mr[];
  const int P = L.count * kin;
  for (int t = threadIdx.x; t < P * d; t += blockDim.x) {
    int r = t % P, c = t / P;
    Mr[t] = M[(size_t)c * ldM + r];
  }
  __syncthreads();
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= N) return;
  double acc[MC];
#pragma unroll
  for (int o = 0; o < MC; ++o) acc[o] = 0.0;
  for (int s = 0; s < L.count; ++s)
    for (int k = 0; k < kin; ++k) {
      const double y = L.ptr[s][(size_t)k * N + l];
      const double* mrow = Mr + s * kin + k;
#pragma unroll
      for (int o = 0; o < MC; ++o)
        if (o < d) acc[o] = fma(y, mrow[o * P], acc[o]);
    }
#pragma unroll
  for (int o = 0; o < MC; ++o)
    if (o < d) out[(size_t)o * N + l] = acc[o];
}

// Sign convention of the DEIM basis: the entry of largest modulus of each
// column (smallest row on ties) is made positive.  One block per column.
__global__ void __launch_bounds__(1024) colsign_kernel(double* __restrict__ A, int N) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  double* a = A + (size_t)blockIdx.x * N;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int l = threadIdx.x; l < N; l += blockDim.x) {
    double v = fabs(a[l]);
    if (v > best) {
      best = v;
      bi = l;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      double v = sv[threadIdx.x + o];
      int vi = si[threadIdx.x + o];
      if (v > sv[threadIdx.x] || (v == sv[threadIdx.x] && vi < si[threadIdx.x])) {
        sv[threadIdx.x] = v;
        si[threadIdx.x] = vi;
      }
    }
    __syncthreads();
  }
  const bool neg = a[si[0]] < 0.0;
  __syncthreads();
  if (neg)
    for (int l = threadIdx.x; l < N; l += blockDim.x) a[l] = -a[l];
}

// Greedy DEIM residual r = psi_k - Psi[:, :k] c and its per-block argmax
// of |r| (smallest index on ties).
__global__ void __launch_bounds__(256) deim_residual_kernel(const double* __restrict__ Psi, int N,
                                                            int k, const double* __restrict__ c,
                                                            double* __restrict__ bval,
                                                            int* __restrict__ bidx) {
  __shared__ double cs[64];
  __shared__ double sv[256];
  __shared__ int si[256];
  for (int t = threadIdx.x; t < k; t += blockDim.x) cs[t] = c[t];
  __syncthreads();
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < N; l += gridDim.x * blockDim.x) {
    double r = Psi[(size_t)k * N + l];
    for (int q = 0; q < k; ++q) r = fma(-Psi[(size_t)q * N + l], cs[q], r);
    const double v = fabs(r);
    if (v > best) {
      best = v;
      bi = l;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      double v = sv[threadIdx.x + o];
      int vi = si[threadIdx.x + o];
      if (v > sv[threadIdx.x] || (v == sv[threadIdx.x] && vi < si[threadIdx.x])) {
        sv[threadIdx.x] = v;
        si[threadIdx.x] = vi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bval[blockIdx.x] = sv[0];
    bidx[blockIdx.x] = si[0];
  }
}

// Column sums of Psi (N x d), partial per block: part[b][j].
__global__ void __launch_bounds__(256) colsum_partial_kernel(const double* __restrict__ Psi, int N,
                                                             int d, double* __restrict__ part) {
  __shared__ double red[8];
  for (int j = 0; j < d; ++j) {
    double s = 0.0;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < N; l += gridDim.x * blockDim.x)
      s += Psi[(size_t)j * N + l];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * d + j] = s;
  }
}

// ---------------------------------------------------------------------------
// Fused gather + projection (eq. grads): g = U~^* G~ (n x p) with
// G~ = F + i v evaluated on the fly and never stored; F = (q/m) e_c at the
// particle's cell, v = Im(U~ Z~).  Lanes are the 64 parameters of a tile
// (blockIdx.y); each wavefront takes one particle row at a time, so the row
// of U~ is wavefront-uniform (scalar loads, no LDS traffic) and the
// projection needs no cross-lane reduction while rows stream.  The field
// rows of the tile sit in LDS.  The eight wavefronts are summed in a fixed
// order; block b writes part[b * rec + c * n + k] and, with want_colsq,
// |G~[:, c]|^2 at part[b * rec + n * p + c].re.  Positions use the operation
// order of the deposit, so both see the same cells.
// ---------------------------------------------------------------------------
template <int NC, bool ET_LDS>
__global__ void __launch_bounds__(512) gather_project_kernel(
    const cplx* __restrict__ U, int N, int n, const cplx* __restrict__ Z, int p, int Nx, int rpb,
    const double* __restrict__ factor, const double* __restrict__ e, double qm,
    const int* __restrict__ active, int rec, int want_colsq, cplx* __restrict__ part) {
  extern __shared__ double smem[];
  double* et = smem;  // [64][Nx] (ET_LDS); after the rows, the wavefront sums
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c0 = blockIdx.y * 64;
  const int c = c0 + lane;
  const int ntc = min(64, p - c0);
  const bool on = (lane < ntc) && (!active || active[c]);
  if (ET_LDS) {
    // the tile's field rows are contiguous: a linear copy, four loads in flight
    const double* es = e + (size_t)c0 * Nx;
    const int tot = ntc * Nx;
    for (int t0 = 0; t0 < tot; t0 += 4 * 512) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + u * 512 + tid;
        v[u] = (t < tot) ? es[t] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + u * 512 + tid;
        if (t < tot) et[t] = qm * v[u];
      }
    }
  }
  cplx z[NC], acc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    z[k] = (on && k < n) ? Z[(size_t)c * n + k] : mk(0.0, 0.0);
    acc[k] = mk(0.0, 0.0);
  }
  const double fac = on ? factor[c] : 1.0;
  double csq = 0.0;
  __syncthreads();
  const int r0 = blockIdx.x * rpb;
  const int r1 = min(N, r0 + rpb);
  if (on) {
    for (int l = r0 + w; l < r1; l += 8) {
      // the padding (k >= n) is zero in u and z: those terms add exact
      // zeros, so the loops run branch-free over NC
      cplx u[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) u[k] = (k < n) ? U[(size_t)k * N + l] : mk(0.0, 0.0);
      double x0 = 0.0, x1 = 0.0, v0 = 0.0, v1 = 0.0;
#pragma unroll
      for (int k = 0; k < NC; k += 2) {
        x0 = fma(u[k].re, z[k].re, x0);
        x0 = fma(-u[k].im, z[k].im, x0);
        v0 = fma(u[k].re, z[k].im, v0);
        v0 = fma(u[k].im, z[k].re, v0);
        x1 = fma(u[k + 1].re, z[k + 1].re, x1);
        x1 = fma(-u[k + 1].im, z[k + 1].im, x1);
        v1 = fma(u[k + 1].re, z[k + 1].im, v1);
        v1 = fma(u[k + 1].im, z[k + 1].re, v1);
      }
      const double v = v0 + v1;
      int j;
      double th;
      cell_of(x0 + x1, fac, Nx, j, th);
      const double F = ET_LDS ? et[lane * Nx + j] : qm * e[(size_t)c * Nx + j];
#pragma unroll
      for (int k = 0; k < NC; ++k) cfmac(acc[k], u[k], mk(F, v));
      csq = fma(F, F, csq);
      csq = fma(v, v, csq);
    }
  }
  // the eight wavefronts in order, through LDS (the field rows are free now)
  __syncthreads();
  cplx* red = reinterpret_cast<cplx*>(smem);                  // [NC][64]
  double* rcs = smem + 2 * NC * 64;                            // [64]
  for (int ww = 0; ww < 8; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int k = 0; k < NC; ++k) red[k * 64 + lane] = (ww == 0) ? acc[k] : cadd(red[k * 64 + lane], acc[k]);
      rcs[lane] = (ww == 0) ? csq : rcs[lane] + csq;
    }
    __syncthreads();
  }
  cplx* pb = part + (size_t)blockIdx.x * rec;
  for (int t = tid; t < ntc * n; t += 512) {
    const int q = t / n, k = t % n;
    pb[(size_t)(c0 + q) * n + k] = red[k * 64 + q];
  }
  if (want_colsq)
    for (int t = tid; t < ntc; t += 512) pb[(size_t)n * p + c0 + t] = mk(rcs[t], 0.0);
}

// C1[o] = sum_b part[b][o] for o < n1, C2[o - n1] = the real part of that sum
// for n1 <= o < nout; blocks summed in a fixed order (one wavefront per output).
__global__ void __launch_bounds__(256) reduce_partials2_kernel(const cplx* __restrict__ part,
                                                               int nkb, int rec, int n1, int nout,
                                                               cplx* __restrict__ C1,
                                                               double* __restrict__ C2) {
  const int lane = threadIdx.x & 63;
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (o >= nout) return;
  double re = 0.0, im = 0.0;
  for (int k = lane; k < nkb; k += 64) {
    const cplx v = part[(size_t)k * rec + o];
    re += v.re;
    im += v.im;
  }
  for (int s = 32; s > 0; s >>= 1) {
    re += __shfl_xor(re, s, 64);
    im += __shfl_xor(im, s, 64);
  }
  if (lane == 0) {
    if (o < n1)
      C1[o] = mk(re, im);
    else
      C2[o - n1] = re;
  }
}

// ---------------------------------------------------------------------------
// Fused gather + basis velocity: out = G~ (-i h Q) + U~ MU (N x n), the
// tangent step xi = h X~ of eq. Xdot in complex form (X~ = -i (G~ Q - U~ g~ Q)),
// with G~ evaluated on the fly (not stored).  One thread per particle row;
// the block walks the parameters in order with the field row of the next
// parameter prefetched into the other half of a two-row LDS buffer.  Q
// (p x n, ld p) and MU (n x n, ld n) as written by the dense kernels.
// ---------------------------------------------------------------------------
template <int NC>
__global__ void __launch_bounds__(256) gather_xi_kernel(
    const cplx* __restrict__ U, int N, int n, const cplx* __restrict__ Z, int p, int Nx,
    const double* __restrict__ factor, const double* __restrict__ e, double qm,
    const cplx* __restrict__ Q, const cplx* __restrict__ MU, double h, cplx* __restrict__ out) {
  extern __shared__ double smem[];
  cplx* Zs = reinterpret_cast<cplx*>(smem);  // [p][NC], zero beyond n
  cplx* Qs = Zs + (size_t)p * NC;            // [p][NC]: -i h Q[c][k], zero beyond n
  cplx* Ms = Qs + (size_t)p * NC;            // [NC][NC]: MU[j][k] at Ms[j * NC + k]
  double* fs = reinterpret_cast<double*>(Ms + NC * NC);  // [p]
  double* tb = fs + p;                       // [2][Nx]: field rows (q/m) e_c
  const int tid = threadIdx.x;
  for (int t = tid; t < p * NC; t += 256) {
    const int c = t / NC, k = t % NC;
    Zs[t] = (k < n) ? Z[(size_t)c * n + k] : mk(0.0, 0.0);
    const cplx qv = (k < n) ? Q[(size_t)k * p + c] : mk(0.0, 0.0);
    Qs[t] = mk(h * qv.im, -h * qv.re);
  }
  for (int t = tid; t < NC * NC; t += 256) {
    const int j = t / NC, k = t % NC;
    Ms[t] = (j < n && k < n) ? MU[(size_t)k * n + j] : mk(0.0, 0.0);
  }
  for (int t = tid; t < p; t += 256) fs[t] = factor[t];
  for (int t = tid; t < Nx; t += 256) tb[t] = qm * e[t];
  const int l = blockIdx.x * 256 + tid;
  const bool valid = l < N;
  cplx u[NC], acc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    u[k] = (valid && k < n) ? U[(size_t)k * N + l] : mk(0.0, 0.0);
    acc[k] = mk(0.0, 0.0);
  }
  __syncthreads();
  // the padding (k >= n) is zero in u, Zs, Qs and Ms: those terms add exact
  // zeros, so the loops run branch-free over NC.  First U~ MU, one row of MU
  // at a time (keeps the register footprint to one row)
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const cplx* mj = Ms + j * NC;
#pragma unroll
    for (int k = 0; k < NC; ++k) cfma(acc[k], u[j], mj[k]);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll 1
  for (int c = 0; c < p; ++c) {
    // prefetch the next field row (Nx <= 1024: at most 4 per thread)
    double pf[4];
    const bool more = c + 1 < p;
#pragma unroll
    for (int u4 = 0; u4 < 4; ++u4) {
      const int t = tid + u4 * 256;
      pf[u4] = (more && t < Nx) ? e[(size_t)(c + 1) * Nx + t] : 0.0;
    }
    const double* te = tb + (c & 1) * Nx;
    const cplx* zc = Zs + c * NC;
    double x0 = 0.0, x1 = 0.0, v0 = 0.0, v1 = 0.0;
#pragma unroll
    for (int k = 0; k < NC; k += 2) {
      const cplx za = zc[k], zb = zc[k + 1];
      x0 = fma(u[k].re, za.re, x0);
      x0 = fma(-u[k].im, za.im, x0);
      v0 = fma(u[k].re, za.im, v0);
      v0 = fma(u[k].im, za.re, v0);
      x1 = fma(u[k + 1].re, zb.re, x1);
      x1 = fma(-u[k + 1].im, zb.im, x1);
      v1 = fma(u[k + 1].re, zb.im, v1);
      v1 = fma(u[k + 1].im, zb.re, v1);
    }
    int j;
    double th;
    cell_of(x0 + x1, fs[c], Nx, j, th);
    const cplx gv = mk(te[j], v0 + v1);
    const cplx* qc = Qs + c * NC;
#pragma unroll
    for (int k = 0; k < NC; ++k) cfma(acc[k], gv, qc[k]);
    if (more) {
      double* tn = tb + ((c + 1) & 1) * Nx;
#pragma unroll
      for (int u4 = 0; u4 < 4; ++u4) {
        const int t = tid + u4 * 256;
        if (t < Nx) tn[t] = qm * pf[u4];
      }
    }
    __syncthreads();
  }
  if (valid) {
#pragma unroll
    for (int k = 0; k < NC; ++k)
      if (k < n) out[(size_t)k * N + l] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
bool fused_gradient_ok(int n) { return n <= 16; }

// register width of the fused kernels: an even count >= n (the position sums
// split into even and odd k, so every even width gives the deposit's cells)
static int fused_nc(int n) {
  if (n <= 4) return 4;
  if (n <= 6) return 6;
  if (n <= 8) return 8;
  if (n <= 12) return 12;
  return 16;
}

void launch_gather_project(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p,
                           int Nx, const double* factor, const double* e, double qm,
                           const int* active, bool want_colsq, cplx* part, size_t part_cap,
                           cplx* g, double* colsq) {
  const int nc = fused_nc(n);
  const int ntile = (p + 63) / 64;
  const int rec = n * p + p;
  // about 256 rows per block (32 per wavefront), at most 1024 blocks,
  // partials within part_cap
  int nb = (N + 255) / 256;
  if (nb > 1024) nb = 1024;
  const int cap = (int)(part_cap / (size_t)rec);
  if (nb > cap) nb = cap;
  if (nb < 1) nb = 1;
  const int rpb = (N + nb - 1) / nb;
  nb = (N + rpb - 1) / rpb;
  const int tw = (p < 64) ? p : 64;
  const size_t et_bytes = (size_t)tw * Nx * sizeof(double);
  const bool et_lds = et_bytes <= 72 * 1024;
  // the wavefront sums reuse the table's space: NC x 64 complex + 64 doubles
  const size_t red_bytes = (size_t)nc * 64 * sizeof(cplx) + 64 * sizeof(double);
  const size_t sh = (et_lds && et_bytes > red_bytes) ? et_bytes : red_bytes;
  dim3 grid(nb, ntile);
#define GPK(NCV, ETV)                                                                          \
  ALLOW_BIG_LDS((gather_project_kernel<NCV, ETV>));                                          \
  hipLaunchKernelGGL((gather_project_kernel<NCV, ETV>), grid, dim3(512), sh, s, U, N, n, Z, p, \
                     Nx, rpb, factor, e, qm, active, rec, want_colsq ? 1 : 0, part)
  if (et_lds) {
    switch (nc) {
      case 4: GPK(4, true); break;
      case 6: GPK(6, true); break;
      case 8: GPK(8, true); break;
      case 12: GPK(12, true); break;
      default: GPK(16, true); break;
    }
  } else {
    switch (nc) {
      case 4: GPK(4, false); break;
      case 6: GPK(6, false); break;
      case 8: GPK(8, false); break;
      case 12: GPK(12, false); break;
      default: GPK(16, false); break;
    }
  }
#undef GPK
  const int nout = want_colsq ? rec : n * p;
  hipLaunchKernelGGL(reduce_partials2_kernel, dim3((nout + 3) / 4), dim3(256), 0, s, part, nb, rec,
                     n * p, nout, g, colsq);
}


void launch_gather_xi(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                      const double* factor, const double* e, double qm, const cplx* Q,
                      const cplx* MU, double h, cplx* out) {
  const int nc = fused_nc(n);
  const size_t sh = (size_t)(2 * p * nc + nc * nc) * sizeof(cplx) + (size_t)(p + 2 * Nx) * sizeof(double);
  dim3 grid((N + 255) / 256);
#define GXK(NCV)                                                                              \
  ALLOW_BIG_LDS(gather_xi_kernel<NCV>);                                                     \
  hipLaunchKernelGGL(gather_xi_kernel<NCV>, grid, dim3(256), sh, s, U, N, n, Z, p, Nx, factor, e, \
                     qm, Q, MU, h, out)
  switch (nc) {
    case 4: GXK(4); break;
    case 6: GXK(6); break;
    case 8: GXK(8); break;
    case 12: GXK(12); break;
    default: GXK(16); break;
  }
#undef GXK
}

void launch_gather_rom(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                       const PicGeom& g, const double* factor, const double* e, double qm,
                       const int* active, bool full, void* out) {
  dim3 grid(g.nrb, (p + g.pt - 1) / g.pt);
  int nc = nc_bucket(n);
  size_t sh = (size_t)g.pt * Nx * sizeof(double) + (size_t)g.pt * nc * sizeof(cplx);
#define GA(NCV, FV)                                                                           \
  ALLOW_BIG_LDS((gather_rom_kernel<NCV, FV>));                                               \
  hipLaunchKernelGGL((gather_rom_kernel<NCV, FV>), grid, dim3(512), sh, s, U, N, n, Z, p, Nx, \
                     g.pt, g.rpb, factor, e, qm, active, out)
  if (full) {
    switch (nc) {
      case 4: GA(4, true); break;
      case 8: GA(8, true); break;
      case 16: GA(16, true); break;
      default: GA(32, true); break;
    }
  } else {
    switch (nc) {
      case 4: GA(4, false); break;
      case 8: GA(8, false); break;
      case 16: GA(16, false); break;
      default: GA(32, false); break;
    }
  }
#undef GA
}

void launch_reconstruct(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p,
                        double* X, double* V) {
  int nc = nc_bucket(n);
  dim3 grid((N + 255) / 256);
  switch (nc) {
    case 4: hipLaunchKernelGGL(reconstruct_kernel<4>, grid, dim3(256), 0, s, U, N, n, Z, p, X, V); break;
    case 8: hipLaunchKernelGGL(reconstruct_kernel<8>, grid, dim3(256), 0, s, U, N, n, Z, p, X, V); break;
    case 16: hipLaunchKernelGGL(reconstruct_kernel<16>, grid, dim3(256), 0, s, U, N, n, Z, p, X, V); break;
    default: hipLaunchKernelGGL(reconstruct_kernel<32>, grid, dim3(256), 0, s, U, N, n, Z, p, X, V); break;
  }
}

void launch_gemm_flags(hipStream_t s, const MatList& A, int a, const MatList& B, int b, int flags,
                       int N, int nkb, cplx* part, cplx* C) {
  // split-K blocks: about 128 rows each, at most 1024, and partials of at
  // most 2^19 complex values (the caller's buffer holds nkb * 64 * 64)
  const int bmax = (b < 64) ? b : 64;
  int cap = (1 << 19) / (a * bmax);
  if (cap > nkb * 64 * 64 / (a * bmax)) cap = nkb * 64 * 64 / (a * bmax);
  nkb = (N + 127) / 128;
  if (nkb > 512) nkb = 512;
  if (nkb > cap) nkb = cap;
  if (nkb < 1) nkb = 1;
  int rk = (N + nkb - 1) / nkb;
  nkb = (N + rk - 1) / rk;
  const bool b_real = flags & GEMM_B_REAL;
  // one staged copy when A and B are the same list of the same kind
  bool same = (a == b) && (((flags & GEMM_A_REAL) != 0) == b_real) && A.count == B.count;
  for (int q = 0; same && q < A.count; ++q)
    same = A.ptr[q] == B.ptr[q] && A.cols[q] == B.cols[q];
  // B is processed in chunks of at most 64 columns (one list entry per chunk)
  for (int b0 = 0; b0 < b; b0 += 64) {
    const int bc = (b - b0 < 64) ? b - b0 : 64;
    MatList Bc = B;
    if (b > 64) {
      Bc.count = 1;
      Bc.cols[0] = bc;
      Bc.ptr[0] = b_real ? reinterpret_cast<const cplx*>(reinterpret_cast<const double*>(B.ptr[0]) +
                                                         (size_t)b0 * N)
                         : B.ptr[0] + (size_t)b0 * N;
    }
    const bool sm_same = same && b <= 64;
    const int nst = sm_same ? a : a + bc;
    // rows per staged chunk: up to 256, within 64 KB of LDS
    int TR = 256;
    while (TR > 32 && nst * TR > 4096) TR >>= 1;
    size_t sh = (size_t)nst * TR * sizeof(cplx);
    if (sh < (size_t)16 * GEMM_RED_LD * sizeof(cplx)) sh = (size_t)16 * GEMM_RED_LD * sizeof(cplx);
    ALLOW_BIG_LDS(gemm_ah_b_kernel);
    hipLaunchKernelGGL(gemm_ah_b_kernel, dim3(nkb), dim3(256), sh, s, A, a, Bc, bc,
                       flags | (sm_same ? GEMM_SAME : 0), N, rk, TR, part);
    int nout = a * bc;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((nout + 3) / 4), dim3(256), 0, s, part, nkb,
                       nout, C + (size_t)b0 * a);
  }
}

void launch_gemm_ah_b(hipStream_t s, const MatList& A, int a, const MatList& B, int b, bool b_real,
                      int N, int nkb, cplx* part, cplx* C) {
  launch_gemm_flags(s, A, a, B, b, b_real ? GEMM_B_REAL : 0, N, nkb, part, C);
}

void launch_rowgemm(hipStream_t s, const RowTerms& T, int N, int m, cplx* out) {
  size_t sh = 0;
  for (int q = 0; q < T.count; ++q) sh += (size_t)T.k[q] * m * sizeof(cplx);
  dim3 grid((N + 255) / 256);
  int mc = nc_bucket(m);
  ALLOW_BIG_LDS(rowgemm_kernel<4>);
  ALLOW_BIG_LDS(rowgemm_kernel<8>);
  ALLOW_BIG_LDS(rowgemm_kernel<16>);
  ALLOW_BIG_LDS(rowgemm_kernel<32>);
  switch (mc) {
    case 4: hipLaunchKernelGGL(rowgemm_kernel<4>, grid, dim3(256), sh, s, T, N, m, out); break;
    case 8: hipLaunchKernelGGL(rowgemm_kernel<8>, grid, dim3(256), sh, s, T, N, m, out); break;
    case 16: hipLaunchKernelGGL(rowgemm_kernel<16>, grid, dim3(256), sh, s, T, N, m, out); break;
    default: hipLaunchKernelGGL(rowgemm_kernel<32>, grid, dim3(256), sh, s, T, N, m, out); break;
  }
}

void launch_deim_gather(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                        const double* factor, const double* e, double qm, const int* idx,
                        const double* w, int d, const int* active, cplx* gF) {
  hipLaunchKernelGGL(deim_gather_kernel, dim3(p), dim3(64), 0, s, U, N, n, Z, p, Nx, factor, e,
                     qm, idx, w, d, active, gF);
}

void launch_snapshot(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, const int* sub,
                     int psub, int Nx, const double* factor, const double* phi, double* Y) {
  int nc = nc_bucket(n);
  dim3 grid((N + 255) / 256);
#define SN(NCV)                                                                               \
  hipLaunchKernelGGL(snapshot_kernel<NCV>, grid, dim3(256), 0, s, U, N, n, Z, sub, psub, Nx, \
                     factor, phi, Y)
  switch (nc) {
    case 4: SN(4); break;
    case 8: SN(8); break;
    case 16: SN(16); break;
    default: SN(32); break;
  }
#undef SN
}

void launch_rowgemm_real(hipStream_t s, const double* const* in, int nin, int kin, int N,
                         const double* M, int ldM, int d, double* out) {
  RealList L{};
  for (int q = 0; q < nin; ++q) L.ptr[q] = in[q];
  L.count = nin;
  size_t sh = (size_t)nin * kin * d * sizeof(double);
  dim3 grid((N + 255) / 256);
  if (d <= 16) {
    ALLOW_BIG_LDS(rowgemm_real_kernel<16>);
    hipLaunchKernelGGL(rowgemm_real_kernel<16>, grid, dim3(256), sh, s, L, kin, N, M, ldM, d, out);
  } else if (d <= 32) {
    ALLOW_BIG_LDS(rowgemm_real_kernel<32>);
    hipLaunchKernelGGL(rowgemm_real_kernel<32>, grid, dim3(256), sh, s, L, kin, N, M, ldM, d, out);
  } else {
    ALLOW_BIG_LDS(rowgemm_real_kernel<64>);
    hipLaunchKernelGGL(rowgemm_real_kernel<64>, grid, dim3(256), sh, s, L, kin, N, M, ldM, d, out);
  }
}

void launch_colsign(hipStream_t s, double* A, int N, int d) {
  hipLaunchKernelGGL(colsign_kernel, dim3(d), dim3(1024), 0, s, A, N);
}

void launch_deim_residual(hipStream_t s, const double* Psi, int N, int k, const double* c,
                          int nblk, double* bval, int* bidx) {
  hipLaunchKernelGGL(deim_residual_kernel, dim3(nblk), dim3(256), 0, s, Psi, N, k, c, bval, bidx);
}

void launch_colsum_partial(hipStream_t s, const double* Psi, int N, int d, int nblk,
                           double* part) {
  hipLaunchKernelGGL(colsum_partial_kernel, dim3(nblk), dim3(256), 0, s, Psi, N, d, part);
}

// ---------------------------------------------------------------------------
// Real product C = A^T B (A: N x a, B: N x b, both real column-major lists,
// a, b <= 64), split over row blocks like gemm_ah_b_kernel.  Output partials
// part[kb][ib * a + ia].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) gemm_real_tn_kernel(RealList A, int ka, int a, RealList B,
                                                           int kbcols, int b, int N, int rk,
                                                           double* __restrict__ part) {
  // tile sums, entry-major with a padded stride (conflict-free writes)
  __shared__ double red[16 * GEMM_RED_LD];
  const int kb = blockIdx.x;
  const int r0 = kb * rk;
  const int r1 = min(N, r0 + rk);
  const int nta = (a + 3) / 4, ntb = (b + 3) / 4, nt = nta * ntb;
  const int R = max(1, 256 / nt);
  const int tid = threadIdx.x;
  const int tile = tid / R, rg = tid % R;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  if (tile < nt) {
    const int ta0 = (tile % nta) * 4, tb0 = (tile / nta) * 4;
    const double* ap[4];
    const double* bp[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ca = ta0 + i, cb = tb0 + i;
      ap[i] = (ca < a) ? A.ptr[ca / ka] + (size_t)(ca % ka) * N : nullptr;
      bp[i] = (cb < b) ? B.ptr[cb / kbcols] + (size_t)(cb % kbcols) * N : nullptr;
    }
    int l = r0 + rg;
    for (; l + R < r1; l += 2 * R) {
      double av[2][4], bv[2][4];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          av[u][i] = ap[i] ? ap[i][l + u * R] : 0.0;
          bv[u][i] = bp[i] ? bp[i][l + u * R] : 0.0;
        }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[u][i], bv[u][j], acc[i][j]);
    }
    for (; l < r1; l += R) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        av[i] = ap[i] ? ap[i][l] : 0.0;
        bv[i] = bp[i] ? bp[i][l] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[(i * 4 + j) * GEMM_RED_LD + tid] = acc[i][j];
  __syncthreads();
  const int nout = a * b;
  for (int o = tid; o < nt * 16; o += blockDim.x) {
    const int tl = o / 16, q = o % 16;
    double sm = 0.0;
#pragma unroll 8
    for (int g = 0; g < R; ++g) sm += red[q * GEMM_RED_LD + tl * R + g];
    const int ia = (tl % nta) * 4 + q / 4, ib = (tl / nta) * 4 + q % 4;
    if (ia < a && ib < b) part[(size_t)kb * nout + (size_t)ib * a + ia] = sm;
  }
}

// Sum the partials of a real product and scatter the a x b result into the
// symmetric P x P matrix S at rows r0.. (and the transpose at columns r0..).
__global__ void __launch_bounds__(256) reduce_gram_block_kernel(const double* __restrict__ part,
                                                                int nkb, int a, int b, int P,
                                                                int r0, double* __restrict__ S) {
  const int lane = threadIdx.x & 63;
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nout = a * b;
  if (o >= nout) return;
  double s = 0.0;
  for (int k = lane; k < nkb; k += 64) s += part[(size_t)k * nout + o];
  for (int w = 32; w > 0; w >>= 1) s += __shfl_xor(s, w, 64);
  if (lane == 0) {
    const int ia = o % a, ib = o / a;
    S[(size_t)ib * P + r0 + ia] = s;   // row r0+ia, column ib
    S[(size_t)(r0 + ia) * P + ib] = s; // transpose
  }
}

void launch_gram_block_real(hipStream_t s, const double* Ynew, const double* const* slots,
                            int nslots, int psub, int N, int r0, int nkb_cap, double* part,
                            double* S) {
  RealList A{}, B{};
  A.ptr[0] = Ynew;
  A.count = 1;
  for (int q = 0; q < nslots; ++q) B.ptr[q] = slots[q];
  B.count = nslots;
  const int a = psub, b = psub * nslots;
  int nkb = (N + 127) / 128;
  if (nkb > 256) nkb = 256;
  const int cap = nkb_cap / (a * b);
  if (nkb > cap) nkb = cap;
  if (nkb < 1) nkb = 1;
  const int rk = (N + nkb - 1) / nkb;
  nkb = (N + rk - 1) / rk;
  hipLaunchKernelGGL(gemm_real_tn_kernel, dim3(nkb), dim3(256), 0, s, A, psub, a, B, psub, b, N, rk,
                     part);
  hipLaunchKernelGGL(reduce_gram_block_kernel, dim3((a * b + 3) / 4), dim3(256), 0, s, part, nkb, a,
                     b, b, r0, S);
}
