// DMD-DEIM hyper-reduction (Sec. 4.1, Sec. 4.2.1 Alg. 1, Sec. 4.3 eq. grHDD,
// Alg. 2) for gfx950: the parameter subset of eq. pSampl, the radial basis
// weights of the DMD coordinates, the DMD of the subset potentials on the
// sliding window, the predicted field tables of every parameter, and the
// per-column fixed point of the coefficients with the DMD-DEIM gradient.
//
// The prediction is formed in real arithmetic.  With Alg. 1's
// B = Y' V S^{-1} and A_tol = W Lambda W^{-1}, the modes are Theta = B W and
// the coordinates Theta^+ Phi = W^{-1} B^+ Phi (B has full column rank), so
//   Re(Theta (Pi * Lambda^s)) = B Re(W Lambda^s W^{-1}) c,  c = B^+ Phi,
// and the radial basis interpolation, linear in the data with real weights,
// acts on c as it would on Pi.  Only M_s = Re(W Lambda^s W^{-1}) needs the
// complex eigendecomposition: it is formed from the complex Schur form
// A_tol = Q T Q^* (Hessenberg reduction, shifted QR), the eigenvectors X of
// T (unit upper triangular) and X^{-1}, as M_s = Re(Q X Lambda^s X^{-1} Q^*).
//
// Small dense steps run in one workgroup each; nothing here is a large
// contraction (N_x x p* T data, r <= 48 modes), so none of it uses MFMA.
#include "common.h"
#include "kernels.h"

namespace {

// (value, index) maximum with ties to the smaller index, over a block of 256
__device__ void block_argmax(double& v, int& i, double* sv, int* si) {
  const int t = threadIdx.x;
  sv[t] = v;
  si[t] = i;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      const double v2 = sv[t + o];
      const int i2 = si[t + o];
      if (v2 > sv[t] || (v2 == sv[t] && i2 < si[t])) {
        sv[t] = v2;
        si[t] = i2;
      }
    }
    __syncthreads();
  }
  v = sv[0];
  i = si[0];
  __syncthreads();
}

__device__ double block_min(double v, double* sv) {
  const int t = threadIdx.x;
  sv[t] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) sv[t] = fmin(sv[t], sv[t + o]);
    __syncthreads();
  }
  v = sv[0];
  __syncthreads();
  return v;
}

__device__ double block_max(double v, double* sv) {
  const int t = threadIdx.x;
  sv[t] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) sv[t] = fmax(sv[t], sv[t + o]);
    __syncthreads();
  }
  v = sv[0];
  __syncthreads();
  return v;
}

__device__ double col_dist(const cplx* __restrict__ Z, int n, int a, int b) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += cabs2(csub(Z[(size_t)a * n + k], Z[(size_t)b * n + k]));
  return sqrt(s);
}

}  // namespace

// ---------------------------------------------------------------------------
// eq. pSampl: greedy farthest-point choice of pstar columns of Z~ (n x p):
// the column of largest norm first, then repeatedly the column farthest from
// its nearest chosen column (ties to the smaller index).  Distances between
// columns of Z~ equal those between reduced states (orthonormal basis).
// One workgroup; dmin: p doubles of scratch.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) subset_select_kernel(const cplx* __restrict__ Z, int n,
                                                            int p, int pstar,
                                                            double* __restrict__ dmin,
                                                            int* __restrict__ S) {
  __shared__ double sv[256];
  __shared__ int si[256];
  const int t = threadIdx.x;
  double best = -1.0;
  int barg = p;
  for (int i = t; i < p; i += 256) {
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += cabs2(Z[(size_t)i * n + k]);
    const double v = sqrt(s);
    if (v > best) {
      best = v;
      barg = i;
    }
  }
  block_argmax(best, barg, sv, si);
  int pick = barg;
  if (t == 0) S[0] = pick;
  for (int i = t; i < p; i += 256) dmin[i] = (i == pick) ? -1.0 : col_dist(Z, n, i, pick);
  __syncthreads();
  for (int k = 1; k < pstar; ++k) {
    best = -2.0;
    barg = p;
    for (int i = t; i < p; i += 256) {
      const double v = dmin[i];
      if (v > best) {
        best = v;
        barg = i;
      }
    }
    block_argmax(best, barg, sv, si);
    pick = barg;
    if (t == 0) S[k] = pick;
    for (int i = t; i < p; i += 256)
      dmin[i] = (i == pick || dmin[i] < 0.0) ? -1.0 : fmin(dmin[i], col_dist(Z, n, i, pick));
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Gaussian radial basis weights (Sec. 4.2.1): every parameter coordinate
// scaled to [0, 1] by the ensemble range (zero range: left at 0), width eps
// = the median distance over the pairs of subset nodes (1 when there is a
// single node), K_kl = exp(-(|x_k - x_l| / eps)^2) factorised by Cholesky,
// and beta_i = K^{-1} phi_i with phi_ik = exp(-(|x_i - x_k| / eps)^2), so
// that a quantity known on the subset interpolates as c_i = sum_k beta_ik c_k;
// subset members take the unit vector of their node.  eta[i * dim + c];
// beta: p x pstar, row i contiguous.  One workgroup; flags[0] |= 64 when K
// is not positive definite.
// ---------------------------------------------------------------------------
constexpr int RBF_MAX_DIM = 8;
constexpr int RBF_MAX_NODES = 64;

__global__ void __launch_bounds__(256) rbf_weights_kernel(const double* __restrict__ eta, int dim,
                                                          int p, const int* __restrict__ S,
                                                          int pstar, int* __restrict__ member,
                                                          double* __restrict__ beta,
                                                          int* __restrict__ flags) {
  __shared__ double sv[256];
  __shared__ double lo[RBF_MAX_DIM], span[RBF_MAX_DIM];
  __shared__ double xs[RBF_MAX_NODES * RBF_MAX_DIM];
  __shared__ double dd[RBF_MAX_NODES * (RBF_MAX_NODES - 1) / 2];
  __shared__ double Kl[RBF_MAX_NODES * RBF_MAX_NODES];
  __shared__ double med[2];
  __shared__ int bad;
  const int t = threadIdx.x;
  for (int c = 0; c < dim; ++c) {
    double mn = INFINITY, mx = -INFINITY;
    for (int i = t; i < p; i += 256) {
      mn = fmin(mn, eta[(size_t)i * dim + c]);
      mx = fmax(mx, eta[(size_t)i * dim + c]);
    }
    mn = block_min(mn, sv);
    mx = block_max(mx, sv);
    if (t == 0) {
      lo[c] = mn;
      span[c] = (mx - mn == 0.0) ? 1.0 : mx - mn;
    }
  }
  if (t == 0) bad = 0;
  for (int i = t; i < p; i += 256) member[i] = -1;
  __syncthreads();
  for (int k = t; k < pstar; k += 256) {
    member[S[k]] = k;
    for (int c = 0; c < dim; ++c)
      xs[k * dim + c] = (eta[(size_t)S[k] * dim + c] - lo[c]) / span[c];
  }
  __syncthreads();
  // pair distances (a < b, row by row) and their median
  const int m = pstar * (pstar - 1) / 2;
  for (int q = t; q < m; q += 256) {
    int a = 0, rem = q;
    while (rem >= pstar - 1 - a) {
      rem -= pstar - 1 - a;
      ++a;
    }
    const int b = a + 1 + rem;
    double s = 0.0;
    for (int c = 0; c < dim; ++c) {
      const double df = xs[a * dim + c] - xs[b * dim + c];
      s += df * df;
    }
    dd[q] = sqrt(s);
  }
  __syncthreads();
  for (int q = t; q < m; q += 256) {
    int rank = 0;
    for (int q2 = 0; q2 < m; ++q2) rank += (dd[q2] < dd[q]) || (dd[q2] == dd[q] && q2 < q);
    if (rank == (m - 1) / 2) med[0] = dd[q];
    if (rank == m / 2) med[1] = dd[q];
  }
  __syncthreads();
  double eps = 1.0;
  if (m > 0) eps = (m & 1) ? med[0] : (med[0] + med[1]) * 0.5;
  // K and its Cholesky factor (lower, in place)
  for (int q = t; q < pstar * pstar; q += 256) {
    const int a = q % pstar, b = q / pstar;
    double s = 0.0;
    for (int c = 0; c < dim; ++c) {
      const double df = xs[a * dim + c] - xs[b * dim + c];
      s += df * df;
    }
    const double r = sqrt(s) / eps;
    Kl[b * pstar + a] = exp(-r * r);
  }
  __syncthreads();
  for (int j = 0; j < pstar; ++j) {
    if (t == 0) {
      double dj = Kl[j * pstar + j];
      for (int k = 0; k < j; ++k) dj -= Kl[k * pstar + j] * Kl[k * pstar + j];
      if (!(dj > 0.0)) {
        bad = 1;
        dj = 1.0;
      }
      Kl[j * pstar + j] = sqrt(dj);
    }
    __syncthreads();
    for (int i = j + 1 + t; i < pstar; i += 256) {
      double v = Kl[j * pstar + i];
      for (int k = 0; k < j; ++k) v -= Kl[k * pstar + i] * Kl[k * pstar + j];
      Kl[j * pstar + i] = v / Kl[j * pstar + j];
    }
    __syncthreads();
  }
  if (t == 0 && bad && flags) atomicOr(flags, 64);
  // beta_i by forward and back substitution in the row of beta itself
  for (int i = t; i < p; i += 256) {
    double* bi = beta + (size_t)i * pstar;
    const int mk_ = member[i];
    if (mk_ >= 0) {
      for (int k = 0; k < pstar; ++k) bi[k] = (k == mk_) ? 1.0 : 0.0;
      continue;
    }
    double xi[RBF_MAX_DIM];
    for (int c = 0; c < dim; ++c) xi[c] = (eta[(size_t)i * dim + c] - lo[c]) / span[c];
    for (int k = 0; k < pstar; ++k) {
      double s = 0.0;
      for (int c = 0; c < dim; ++c) {
        const double df = xi[c] - xs[k * dim + c];
        s += df * df;
      }
      const double r = sqrt(s) / eps;
      double v = exp(-r * r);
      for (int q = 0; q < k; ++q) v -= Kl[q * pstar + k] * bi[q];
      bi[k] = v / Kl[k * pstar + k];
    }
    for (int k = pstar - 1; k >= 0; --k) {
      double v = bi[k];
      for (int q = k + 1; q < pstar; ++q) v -= Kl[k * pstar + q] * bi[q];
      bi[k] = v / Kl[k * pstar + k];
    }
  }
}

// ---------------------------------------------------------------------------
// Columns of a p x Nx row-major grid (selected by cols, or the first k) into
// a k x Nx block: the subset potentials of one window level.
// ---------------------------------------------------------------------------
__global__ void grid_rows_kernel(const double* __restrict__ src, const int* __restrict__ cols,
                                 int k, int Nx, double* __restrict__ dst) {
  const int q = blockIdx.x;
  const int c = cols ? cols[q] : q;
  for (int j = threadIdx.x; j < Nx; j += blockDim.x)
    dst[(size_t)q * Nx + j] = src[(size_t)c * Nx + j];
}

// columns S of Z~ (n x p) into a compact n x k block
__global__ void gather_zcols_kernel(const cplx* __restrict__ Z, int n, const int* __restrict__ S,
                                    int k, cplx* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * k) return;
  const int q = t / n, a = t - q * n;
  out[t] = Z[(size_t)S[q] * n + a];
}

// ---------------------------------------------------------------------------
// The window matrices of eq. DMD_potential_Y_time_parameter: Y (N_x x P,
// P = p* T) holds for every subset parameter q its first T window levels,
// Y' the last T, parameter-major (column q T + t is level t, resp. t + 1).
// Level t sits in ring slot (base + t) mod nslots, a p* x N_x block.
// ---------------------------------------------------------------------------
__global__ void dmd_window_kernel(const double* __restrict__ ring, int nslots, int base, int pstar,
                                  int T, int Nx, double* __restrict__ Y, double* __restrict__ Yp) {
  const int col = blockIdx.x;
  const int q = col / T, t = col - q * T;
  const double* l0 = ring + (size_t)((base + t) % nslots) * pstar * Nx + (size_t)q * Nx;
  const double* l1 = ring + (size_t)((base + t + 1) % nslots) * pstar * Nx + (size_t)q * Nx;
  for (int j = threadIdx.x; j < Nx; j += blockDim.x) {
    Y[(size_t)col * Nx + j] = l0[j];
    Yp[(size_t)col * Nx + j] = l1[j];
  }
}

// Reflection of one column held in LDS by one thread: col[k:Nx] -=
// tau (v^T col[k:Nx]) v with v = vk[k:Nx].  Rows in chunks of 8 whose loads
// are issued together and unpredicated (the region is followed by 8 doubles
// of slack; rows past Nx are masked by selects, not branches), so the
// thread waits for LDS once per chunk, not once per row.
__device__ __forceinline__ void reflect_col_lds(const double* vk, double* col, int k, int Nx,
                                                double tk) {
  double d = 0.0;
  for (int i0 = k; i0 < Nx; i0 += 8) {
    double wv[8], cv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      wv[u] = vk[i0 + u];
      cv[u] = col[i0 + u];
    }
    // (the rows past Nx hold padding or the next column, possibly never
    // written: the accumulation itself is selected, so no product of them
    // reaches d)
#pragma unroll
    for (int u = 0; u < 8; ++u) d = (i0 + u < Nx) ? fma(wv[u], cv[u], d) : d;
  }
  const double f = tk * d;
  for (int i0 = k; i0 < Nx; i0 += 8) {
    double wv[8], cv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      wv[u] = vk[i0 + u];
      cv[u] = col[i0 + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u < Nx) col[i0 + u] = fma(-f, wv[u], cv[u]);
  }
}

// ---------------------------------------------------------------------------
// Householder QR of an Nx x P matrix W (column-major, leading dimension ld,
// in place), one
// workgroup of 256: reflector k (k < min(Nx, P)) is stored below the
// diagonal with its head in W[k, k] replaced by v_0, alpha_k (the diagonal
// of R) in alpha[k] and 2 / v^T v in tau[k]; R above the diagonal stays in
// W.  Every further column (and the ncx columns of X, Nx x ncx with the same
// leading dimension, when given)
// is updated either by one thread that runs down its rows (ByThread: W in
// LDS, followed by 8 doubles of slack; no cross-lane reduction, loads in
// chunks of 8) or by the wavefront
// that owns it (column j by wave j mod 4, coalesced rows: W in global).
// ---------------------------------------------------------------------------
template <bool ByThread>
__device__ void householder_qr(double* W, int Nx, int ld, int P, double* alpha, double* tau,
                               double* X, int ncx, double* red) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int mq = min(Nx, P);
  for (int k = 0; k < mq; ++k) {
    double* wk = W + (size_t)k * ld;
    double s = 0.0;
    for (int i = k + t; i < Nx; i += 256) s += wk[i] * wk[i];
    const double nrm2 = block_sum(s, red);
    const double x0 = wk[k];
    const double nrm = sqrt(nrm2);
    const double al = (x0 >= 0.0) ? -nrm : nrm;
    const double v0 = x0 - al;
    const double vtv = nrm2 - x0 * x0 + v0 * v0;
    const double tk = (nrm > 0.0 && vtv > 0.0) ? 2.0 / vtv : 0.0;
    __syncthreads();
    if (t == 0) {
      alpha[k] = (nrm > 0.0) ? al : x0;
      tau[k] = tk;
      wk[k] = v0;
    }
    __syncthreads();
    if (tk != 0.0) {
      const int ntot = (P - k - 1) + ncx;
      if (ByThread) {
        // (W in LDS with 8 doubles of slack past its last column)
        for (int c = t; c < ntot; c += 256) {
          double* col = (c < P - k - 1) ? W + (size_t)(k + 1 + c) * ld
                                        : X + (size_t)(c - (P - k - 1)) * ld;
          reflect_col_lds(wk, col, k, Nx, tk);
        }
      } else {
        for (int c = wv; c < ntot; c += 4) {
          double* col = (c < P - k - 1) ? W + (size_t)(k + 1 + c) * ld
                                        : X + (size_t)(c - (P - k - 1)) * ld;
          double d = 0.0;
          for (int i = k + lane; i < Nx; i += 64) d = fma(wk[i], col[i], d);
          d = wave_sum64(d);
          const double f = tk * d;
          for (int i = k + lane; i < Nx; i += 64) col[i] = fma(-f, wk[i], col[i]);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Alg. 1, step 1: the truncated SVD of Y (N_x x P, P <= 64) by Householder
// QR (work copy W) and one-sided Jacobi on the columns of R (m x P, m =
// min(N_x, P), in LDS) with the rotations accumulated, or on those of R^T
// when the window is wider than the grid (fewer, longer columns); no Gram
// of Y is formed.  With R: V = the rotations, U = Q [R V S^{-1}; 0] from the
// rotated columns, which the stopping rule leaves orthogonal to working
// precision.  With R^T (R^T G = V S): V = the rotated columns over their
// norms, U = Q [G; 0].  (U = Y V S^{-1}
// would lose orthogonality between the columns of small singular values,
// by about eps s_1 / s_j, and A_tol = U^T B with it.)  Output sorted by
// decreasing singular value: sig (P), V (P x P, ld P), the retained count
// r = #{sig_j > tol sig_1} in rout[0] and U (N_x x r, ld Nx).  flags[0] |=
// 128 when Jacobi did not settle in 60 sweeps or Y is zero.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) dmd_svd_kernel(double* __restrict__ W, int Nx, int P,
                                                      double tol, double* __restrict__ sig,
                                                      double* __restrict__ Vout,
                                                      int* __restrict__ rout,
                                                      double* __restrict__ Uout,
                                                      int* __restrict__ flags) {
  __shared__ double red[8];
  __shared__ double alpha[64], tau[64];
  __shared__ double sv[64];
  __shared__ int rot, rkeep;
  __shared__ int perm[64];
  extern __shared__ double jsm[];
  // column j at Rs[j * JS]: the stride of 65 doubles puts element i of the
  // columns that concurrent pair groups rotate in different LDS banks
  constexpr int JS = 65;
  double* Rs = jsm;
  double* Vs = jsm + 64 * JS;
  const int t = threadIdx.x;
  // the QR in LDS when the window fits (ldl P <= 8192 doubles, ldl = N_x
  // rounded up to odd so that the columns that the threads of a wavefront
  // walk down fall in different banks): every reflection then waits on LDS,
  // not on global loads
  const int ldl = Nx | 1;
  const bool lw = ldl * P + 8 <= 8192;
  const int ldq = lw ? ldl : Nx;
  double* Wl = jsm + 2 * 64 * JS;
  if (lw) {
    for (int q = t; q < Nx * P; q += 256) {
      const int j = q / Nx, i = q - j * Nx;
      Wl[j * ldl + i] = W[q];
    }
    __syncthreads();
    householder_qr<true>(Wl, Nx, ldl, P, alpha, tau, nullptr, 0, red);
  } else {
    householder_qr<false>(W, Nx, Nx, P, alpha, tau, nullptr, 0, red);
  }
  const double* Wq = lw ? Wl : W;
  const int m = min(Nx, P);
  // Jacobi on the columns of R (m x P) when m = P, on those of R^T (P x m)
  // when the window is wider than the grid (m < P): C columns of length ell,
  // the rotations accumulated in G (C x C).  R (upper trapezoidal): R[i][j]
  // = W[j Nx + i] above the diagonal, alpha[i] on it.
  const bool wide = m < P;
  const int C = wide ? m : P, ell = wide ? P : m;
  for (int q = t; q < 64 * 64; q += 256) {
    const int j = q >> 6, i = q & 63;
    double v = 0.0;
    if (j < C && i < ell) {
      const int ri = wide ? j : i, rj = wide ? i : j;  // the entry R[ri][rj]
      v = (ri < rj) ? Wq[(size_t)rj * ldq + ri] : (ri == rj ? alpha[ri] : 0.0);
    }
    Rs[j * JS + i] = v;
    Vs[j * JS + i] = (i == j && j < C) ? 1.0 : 0.0;
  }
  __syncthreads();
  // columns at rounding level (|col|^2 below (1e-15 |R|_F)^2) take part in
  // no rotation: their mutual rounding noise never settles
  double fr = 0.0;
  for (int q = t; q < 64 * 64; q += 256) {
    const double v = Rs[(q >> 6) * JS + (q & 63)];
    fr = fma(v, v, fr);
  }
  const double frob2 = block_sum(fr, red);
  const double tiny = 1e-30 * frob2;
  // round-robin pairs (circle method) over C2 = C rounded up to even; a
  // pair with the padding column is skipped
  const int C2 = C + (C & 1);
  const int g = t >> 3, sub = t & 7;
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    if (t == 0) rot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < C2 - 1; ++rnd) {
      // (the 8 lanes of a pair group sit in one DPP row half: every lane of
      // the group takes part in the sums below, also when its pair is idle)
      int ia = g - 1 + rnd, ib = C2 - 2 - g + rnd;
      ia = (ia >= C2 - 1) ? ia - (C2 - 1) : ia;
      ib = (ib >= C2 - 1) ? ib - (C2 - 1) : ib;
      ia = (g == 0) ? 0 : ia + 1;
      ib = ib + 1;
      const bool act = g < C2 / 2 && ia < C && ib < C;
      {
        // the lane's elements of both columns (and of G) in registers: one
        // batch of loads, the sums, the rotation, one batch of stores
        // (unpredicated: entries past ell of a column of R and past C of
        // one of G are zero and stay zero under the rotations, and an idle
        // group reads column 0 and writes nothing)
        const int a = act ? min(ia, ib) : 0, b = act ? max(ia, ib) : 0;
        double xa[8], xb[8], ga_[8], gb_[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = sub + 8 * u;
          xa[u] = Rs[a * JS + i];
          xb[u] = Rs[b * JS + i];
          ga_[u] = Vs[a * JS + i];
          gb_[u] = Vs[b * JS + i];
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          al = fma(xa[u], xa[u], al);
          be = fma(xb[u], xb[u], be);
          ga = fma(xa[u], xb[u], ga);
        }
        // sums over the 8 lanes of the group by DPP butterflies
        al += bfly64<0>(al);
        be += bfly64<0>(be);
        ga += bfly64<0>(ga);
        al += bfly64<1>(al);
        be += bfly64<1>(be);
        ga += bfly64<1>(ga);
        al += bfly64<2>(al);
        be += bfly64<2>(be);
        ga += bfly64<2>(ga);
        if (act && ga != 0.0 && al > tiny && be > tiny && ga * ga > 1e-30 * (al * be)) {
          // tan of the rotation, the root of smaller modulus of t^2 + 2 zeta t
          // - 1 = 0 with zeta = (be - al) / (2 ga): t = sign(d) 2ga / (|d| +
          // hypot(d, 2ga)), d = be - al (t = +-1 when d = 0)
          const double d = be - al, g2 = 2.0 * ga;
          const double tt = ((d >= 0.0) ? g2 : -g2) / (fabs(d) + sqrt(fma(d, d, g2 * g2)));
          const double c = 1.0 / sqrt(fma(tt, tt, 1.0)), s = c * tt;
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int i = sub + 8 * u;
            Rs[a * JS + i] = c * xa[u] - s * xb[u];
            Rs[b * JS + i] = s * xa[u] + c * xb[u];
            Vs[a * JS + i] = c * ga_[u] - s * gb_[u];
            Vs[b * JS + i] = s * ga_[u] + c * gb_[u];
          }
          if (sub == 0) rot = 1;
        }
      }
      __syncthreads();
    }
    const int any = rot;
    __syncthreads();
    if (!any) break;
  }
  if (t < C) {
    double s = 0.0;
    for (int i = 0; i < ell; ++i) s = fma(Rs[t * JS + i], Rs[t * JS + i], s);
    sv[t] = sqrt(s);
  }
  __syncthreads();
  // right vectors: the rotations (R) or the rotated columns over their norms (R^T)
  if (t < C) {
    int rank = 0;
    for (int j = 0; j < C; ++j) rank += (sv[j] > sv[t]) || (sv[j] == sv[t] && j < t);
    sig[rank] = sv[t];
    for (int i = 0; i < P; ++i)
      Vout[(size_t)rank * P + i] = wide ? (sv[t] > 0.0 ? Rs[t * JS + i] / sv[t] : 0.0)
                                        : Vs[t * JS + i];
  }
  for (int k = C + t; k < P; k += 256) sig[k] = 0.0;
  if (t == 0) {
    double smax = 0.0;
    for (int j = 0; j < C; ++j) smax = fmax(smax, sv[j]);
    int r = 0;
    for (int j = 0; j < C; ++j) r += sv[j] > tol * smax;
    rout[0] = r;
    rkeep = r;
    if ((sweep == 60 || smax == 0.0) && flags) atomicOr(flags, 128);
  }
  __syncthreads();
  // U: the small left vectors (the rotated columns over their norms for R,
  // the rotations for R^T), padded to N_x rows, then Q = H_0 ... H_{m-1}
  // applied from the last reflector to the first.  With the reflectors in
  // LDS the r columns are staged in the half of the Jacobi storage that the
  // right vectors have been read from (ld ldl), column c of U is run by
  // thread c, and U is written out at the end; otherwise U is formed in
  // global memory, column c by wavefront c mod 4.
  const int r = rkeep;
  if (t < C) {
    int rank = 0;
    for (int jj = 0; jj < C; ++jj) rank += (sv[jj] > sv[t]) || (sv[jj] == sv[t] && jj < t);
    perm[t] = rank;
  }
  __syncthreads();
  const double* src = wide ? Vs : Rs;
  const bool lu = lw && r * ldl + 8 <= 64 * JS;
  double* Ul = wide ? Rs : Vs;
  for (int q = t; q < C * Nx; q += 256) {
    const int j = q / Nx, i = q - j * Nx;
    const int rank = perm[j];
    if (rank < r) {
      const double v = (i < m) ? (wide ? src[j * JS + i] : src[j * JS + i] / sv[j]) : 0.0;
      if (lu)
        Ul[rank * ldl + i] = v;
      else
        Uout[(size_t)rank * Nx + i] = v;
    }
  }
  __threadfence_block();
  __syncthreads();
  if (lu) {
    // (Ul ends at least 8 doubles before the end of its half of the Jacobi
    // storage or runs into Wl; Wl has 8 doubles of slack)
    for (int c = t; c < r; c += 256) {
      double* u = Ul + c * ldl;
      for (int k = m - 1; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;
        reflect_col_lds(Wl + k * ldl, u, k, Nx, tk);
      }
    }
    __syncthreads();
    for (int q = t; q < r * Nx; q += 256) {
      const int c = q / Nx, i = q - c * Nx;
      Uout[q] = Ul[c * ldl + i];
    }
  } else {
    const int lane = t & 63, wv = t >> 6;
    for (int c = wv; c < r; c += 4) {
      double* u = Uout + (size_t)c * Nx;
      for (int k = m - 1; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;
        const double* vk = Wq + (size_t)k * ldq;
        double d = 0.0;
        for (int i = k + lane; i < Nx; i += 64) d = fma(vk[i], u[i], d);
        d = wave_sum64(d);
        const double f = tk * d;
        for (int i = k + lane; i < Nx; i += 64) u[i] = fma(-f, vk[i], u[i]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Alg. 1, step 2: with V_r S_r^{-1} (the retained right vectors, each over
// its singular value), B = Y' V_r S_r^{-1} (N_x x r, ld Nx) and A_tol =
// U_r^T B (r x r, ld r) with the left vectors U_r of the SVD kernel.  One
// workgroup of 256.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) dmd_form_kernel(const double* __restrict__ Yp, int Nx,
                                                       int P, const double* __restrict__ sig,
                                                       const double* __restrict__ V,
                                                       const int* __restrict__ rin,
                                                       double* __restrict__ B,
                                                       const double* __restrict__ U,
                                                       double* __restrict__ A) {
  __shared__ double Vs[64 * 64];
  const int r = rin[0];
  const int t = threadIdx.x;
  for (int q = t; q < P * r; q += 256) {
    const int a = q / P;
    Vs[q] = V[q] / sig[a];
  }
  __syncthreads();
  for (int q = t; q < Nx * r; q += 256) {
    const int a = q / Nx, j = q - a * Nx;
    double sb = 0.0;
    for (int c = 0; c < P; ++c) sb = fma(Yp[(size_t)c * Nx + j], Vs[a * P + c], sb);
    B[q] = sb;
  }
  __threadfence_block();
  __syncthreads();
  for (int q = t; q < r * r; q += 256) {
    const int b = q / r, a = q - b * r;
    double s = 0.0;
    for (int j = 0; j < Nx; ++j) s = fma(U[(size_t)a * Nx + j], B[(size_t)b * Nx + j], s);
    A[q] = s;
  }
}

// ---------------------------------------------------------------------------
// Alg. 1, step 3, and the half-step growth of eq. DMD_approx_potential_subset:
// M = Re(W Lambda^{1/2} W^{-1}) for A_tol = W Lambda W^{-1} (r x r real,
// r <= 48, principal square root), formed from the complex Schur form
// A_tol = Q T Q^* as Re(Q X Lambda^{1/2} X^{-1} Q^*) with X the unit upper
// triangular eigenvectors of T.  Hessenberg reduction by Householder, then
// single-shift QR sweeps (Wilkinson shift, exceptional shift every 10
// sweeps without deflation) with Givens rotations.  One wavefront: lane j
// owns column j (row operations) or row j (column operations).  Dynamic
// LDS: H, Q, X, Y (r x r complex each, ld r).  Output M (r x r, ld r) and
// the eigenvalues lam (r).  flags[0] |= 256 when QR did not converge in 40 r
// sweeps.
// ---------------------------------------------------------------------------
constexpr int DMD_MAX_R = 48;

__device__ inline cplx cdivx(cplx a, cplx b) {
  // a / b with scaling (Smith)
  if (fabs(b.re) >= fabs(b.im)) {
    const double q = b.im / b.re, den = b.re + b.im * q;
    return mk((a.re + a.im * q) / den, (a.im - a.re * q) / den);
  }
  const double q = b.re / b.im, den = b.re * q + b.im;
  return mk((a.re * q + a.im) / den, (a.im * q - a.re) / den);
}

__device__ inline double cabs1(cplx a) { return fabs(a.re) + fabs(a.im); }

__device__ inline cplx csqrt_principal(cplx z) {
  const double a = z.re, b = z.im;
  const double m = hypot(a, b);
  if (m == 0.0) return mk(0.0, 0.0);
  if (a >= 0.0) {
    const double re = sqrt(0.5 * (m + a));
    return mk(re, b / (2.0 * re));
  }
  const double im = copysign(sqrt(0.5 * (m - a)), b);
  return mk(b / (2.0 * im), im);
}

__global__ void __launch_bounds__(64) dmd_eig_kernel(const double* __restrict__ A,
                                                     const int* __restrict__ rin,
                                                     double* __restrict__ Mout,
                                                     cplx* __restrict__ lam_out,
                                                     int* __restrict__ flags) {
  extern __shared__ cplx dsm[];
  __shared__ cplx vv[DMD_MAX_R];
  __shared__ cplx lam[DMD_MAX_R];
  const int r = rin[0];
  const int L = threadIdx.x;
  cplx* H = dsm;
  cplx* Q = dsm + (size_t)r * r;
  cplx* X = Q + (size_t)r * r;
  cplx* Yi = X + (size_t)r * r;
#define HH(i, j) H[(size_t)(j) * r + (i)]
#define QQ(i, j) Q[(size_t)(j) * r + (i)]
  for (int q = L; q < r * r; q += 64) {
    H[q] = mk(A[q], 0.0);
    Q[q] = mk((q % r) == (q / r) ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // Hessenberg reduction: for column k, the reflector of H[k+1:, k]
  for (int k = 0; k + 2 < r; ++k) {
    double nrm2 = 0.0;
    for (int i = k + 1; i < r; ++i) nrm2 += cabs2(HH(i, k));
    const double nrm = sqrt(nrm2);
    const cplx x0 = HH(k + 1, k);
    const double ax0 = sqrt(cabs2(x0));
    if (nrm == 0.0) continue;
    const cplx ph = (ax0 > 0.0) ? mk(x0.re / ax0, x0.im / ax0) : mk(1.0, 0.0);
    const cplx al = mk(-ph.re * nrm, -ph.im * nrm);  // alpha = -e^{i arg x0} |x|
    // v = x - alpha e_1 (held by the lanes of rows k+1 .. r-1)
    if (L >= k + 1 && L < r) vv[L] = (L == k + 1) ? csub(x0, al) : HH(L, k);
    __syncthreads();
    double vtv = 0.0;
    for (int i = k + 1; i < r; ++i) vtv += cabs2(vv[i]);
    const double tk = 2.0 / vtv;
    // left: H[k+1:, j] -= tk v (v^* H[k+1:, j]), lane = column j
    if (L < r) {
      cplx d = mk(0.0, 0.0);
      for (int i = k + 1; i < r; ++i) cfmac(d, vv[i], HH(i, L));
      d = cscale(d, tk);
      for (int i = k + 1; i < r; ++i) HH(i, L) = csub(HH(i, L), cmul(vv[i], d));
    }
    __syncthreads();
    // right: H[i, k+1:] -= tk (H[i, k+1:] v) v^*, and the same on Q; lane = row i
    if (L < r) {
      cplx d = mk(0.0, 0.0), e = mk(0.0, 0.0);
      for (int j = k + 1; j < r; ++j) {
        cfma(d, HH(L, j), vv[j]);
        cfma(e, QQ(L, j), vv[j]);
      }
      d = cscale(d, tk);
      e = cscale(e, tk);
      for (int j = k + 1; j < r; ++j) {
        HH(L, j) = csub(HH(L, j), cmulc(vv[j], d));
        QQ(L, j) = csub(QQ(L, j), cmulc(vv[j], e));
      }
    }
    __syncthreads();
    if (L > k + 1 && L < r) HH(L, k) = mk(0.0, 0.0);
    __syncthreads();
  }
  // shifted QR on the Hessenberg matrix
  int hi = r - 1, its = 0, total = 0;
  const double eps = 2.220446049250313e-16;
  bool failed = false;
  while (hi > 0) {
    // the active block [lo, hi]: the largest lo with H[lo, lo-1] negligible
    int lo = hi;
    while (lo > 0) {
      const double sub = cabs1(HH(lo, lo - 1));
      double scale = cabs1(HH(lo, lo)) + cabs1(HH(lo - 1, lo - 1));
      if (scale == 0.0) scale = 1.0;
      if (sub <= eps * scale) break;
      --lo;
    }
    __syncthreads();
    if (lo > 0 && L == 0) HH(lo, lo - 1) = mk(0.0, 0.0);
    __syncthreads();
    if (lo == hi) {
      --hi;
      its = 0;
      continue;
    }
    if (++total > 40 * r) {
      failed = true;
      break;
    }
    ++its;
    // shift: the eigenvalue of the trailing 2 x 2 nearer H[hi, hi]
    // (Wilkinson), or an exceptional one every 10 sweeps
    cplx mu;
    if (its % 10 == 0) {
      const double ex = cabs1(HH(hi, hi - 1)) + (hi >= 2 ? cabs1(HH(hi - 1, hi - 2)) : 0.0);
      mu = cadd(HH(hi, hi), mk(0.75 * ex, 0.0));
    } else {
      const cplx a = HH(hi - 1, hi - 1), b = HH(hi - 1, hi), c = HH(hi, hi - 1), d = HH(hi, hi);
      const cplx hf = cscale(csub(a, d), 0.5);
      const cplx disc = csqrt_principal(cadd(cmul(hf, hf), cmul(b, c)));
      const cplx m1 = cadd(hf, disc), m2 = csub(hf, disc);
      // d - b c / (hf +- disc): the root nearer d
      const cplx den = (cabs2(m1) >= cabs2(m2)) ? m1 : m2;
      mu = (cabs2(den) > 0.0) ? csub(d, cdivx(cmul(b, c), den)) : d;
    }
    cplx x = csub(HH(lo, lo), mu), y = HH(lo + 1, lo);
    for (int k = lo; k < hi; ++k) {
      if (k > lo) {
        x = HH(k, k - 1);
        y = HH(k + 1, k - 1);
      }
      // G = [c s; -conj(s) c] with G [x; y] = [rho; 0], c real
      const double ax = sqrt(cabs2(x)), ay = sqrt(cabs2(y));
      double c;
      cplx s;
      if (ay == 0.0) {
        c = 1.0;
        s = mk(0.0, 0.0);
      } else if (ax == 0.0) {
        c = 0.0;
        s = mk(y.re / ay, -y.im / ay);  // conj(y) / |y|
      } else {
        const double nr = hypot(ax, ay);
        c = ax / nr;
        // s = (x / |x|) conj(y) / nr
        const cplx ux = mk(x.re / ax, x.im / ax);
        s = cscale(cmul(ux, cconj(y)), 1.0 / nr);
      }
      __syncthreads();
      // rows k, k+1 (columns from max(lo, k-1) to the end: the whole Schur form)
      const int j0 = (k > lo) ? k - 1 : lo;
      if (L >= j0 && L < r) {
        const cplx h1 = HH(k, L), h2 = HH(k + 1, L);
        HH(k, L) = cadd(cscale(h1, c), cmul(s, h2));
        HH(k + 1, L) = csub(cscale(h2, c), cmulc(s, h1));
      }
      __syncthreads();
      // columns k, k+1 (rows 0 .. min(k+2, hi)), and Q's columns
      const int i1 = min(k + 2, hi);
      if (L <= i1) {
        const cplx h1 = HH(L, k), h2 = HH(L, k + 1);
        HH(L, k) = cadd(cscale(h1, c), cmulc(s, h2));
        HH(L, k + 1) = csub(cscale(h2, c), cmul(s, h1));
      }
      if (L < r) {
        const cplx q1 = QQ(L, k), q2 = QQ(L, k + 1);
        QQ(L, k) = cadd(cscale(q1, c), cmulc(s, q2));
        QQ(L, k + 1) = csub(cscale(q2, c), cmul(s, q1));
      }
      __syncthreads();
      if (k > lo && L == 0) HH(k + 1, k - 1) = mk(0.0, 0.0);
      __syncthreads();
    }
  }
  if (failed && L == 0 && flags) atomicOr(flags, 256);
  if (L < r) lam[L] = HH(L, L);
  __syncthreads();
  // eigenvectors of T (unit upper triangular X, column k by lane k)
  double tn = 0.0;
  for (int q = 0; q < r * r; ++q) tn = fmax(tn, cabs1(H[q]));
  const double smin = fmax(eps * tn, 1e-300);
  if (L < r) {
    const int k = L;
    for (int j = r - 1; j > k; --j) X[(size_t)k * r + j] = mk(0.0, 0.0);
    X[(size_t)k * r + k] = mk(1.0, 0.0);
    for (int j = k - 1; j >= 0; --j) {
      cplx s = mk(0.0, 0.0);
      for (int l = j + 1; l <= k; ++l) cfma(s, HH(j, l), X[(size_t)k * r + l]);
      cplx d = csub(lam[j], lam[k]);
      if (cabs1(d) < smin) d = mk(smin, 0.0);
      X[(size_t)k * r + j] = cdivx(mk(-s.re, -s.im), d);
    }
  }
  __syncthreads();
  // Y = X^{-1} (unit upper triangular, column k by lane k)
  if (L < r) {
    const int k = L;
    for (int j = r - 1; j > k; --j) Yi[(size_t)k * r + j] = mk(0.0, 0.0);
    Yi[(size_t)k * r + k] = mk(1.0, 0.0);
    for (int j = k - 1; j >= 0; --j) {
      cplx s = mk(0.0, 0.0);
      for (int l = j + 1; l <= k; ++l) cfma(s, X[(size_t)l * r + j], Yi[(size_t)k * r + l]);
      Yi[(size_t)k * r + j] = mk(-s.re, -s.im);
    }
  }
  __syncthreads();
  // F = X diag(lam^{1/2}) Y into H (upper triangular, column k by lane k)
  if (L < r) {
    const int k = L;
    for (int i = 0; i < r; ++i) {
      cplx s = mk(0.0, 0.0);
      if (i <= k)
        for (int l = i; l <= k; ++l)
          cfma(s, cmul(X[(size_t)l * r + i], csqrt_principal(lam[l])), Yi[(size_t)k * r + l]);
      HH(i, k) = s;
    }
  }
  __syncthreads();
  // W1 = Q F into X (row i by lane i), then M = Re(W1 Q^*)
  if (L < r) {
    for (int k = 0; k < r; ++k) {
      cplx s = mk(0.0, 0.0);
      for (int l = 0; l <= k; ++l) cfma(s, QQ(L, l), HH(l, k));
      X[(size_t)k * r + L] = s;
    }
  }
  __syncthreads();
  if (L < r) {
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int k = 0; k < r; ++k) {
        const cplx w = X[(size_t)k * r + L], q = QQ(j, k);
        s = fma(w.re, q.re, s);
        s = fma(w.im, q.im, s);  // Re(w conj(q))
      }
      Mout[(size_t)j * r + L] = s;
    }
    lam_out[L] = lam[L];
  }
#undef HH
#undef QQ
}

// ---------------------------------------------------------------------------
// Coordinates of the subset potentials: c_q = B^+ Phi^q_{tau-1} (r x p*,
// ld r) by Householder QR of B (work copy Wb, N_x x r) applied to the p*
// last-level columns (work copy Wf, N_x x p*) and back substitution; and
// BM = B M (N_x x r, ld Nx) for the half-step prediction.  One workgroup of
// 256.  flags[0] |= 512 when B is numerically rank deficient.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) dmd_coords_kernel(const double* __restrict__ B,
                                                         const double* __restrict__ M,
                                                         const int* __restrict__ rin, int Nx,
                                                         int pstar, double* __restrict__ Wb,
                                                         double* __restrict__ Wf,
                                                         double* __restrict__ C,
                                                         double* __restrict__ BM,
                                                         int* __restrict__ flags) {
  __shared__ double red[8];
  __shared__ double alpha[64], tau[64];
  const int r = rin[0];
  const int t = threadIdx.x;
  for (int q = t; q < Nx * r; q += 256) Wb[q] = B[q];
  __threadfence_block();
  __syncthreads();
  householder_qr<false>(Wb, Nx, Nx, r, alpha, tau, Wf, pstar, red);
  double amax = 0.0;
  for (int k = 0; k < r; ++k) amax = fmax(amax, fabs(alpha[k]));
  bool bad = false;
  for (int k = 0; k < r; ++k) bad |= !(fabs(alpha[k]) > 1e-14 * amax);
  if (t == 0 && bad && flags) atomicOr(flags, 512);
  for (int q = t; q < pstar; q += 256) {
    const double* f = Wf + (size_t)q * Nx;
    double* c = C + (size_t)q * r;
    for (int k = r - 1; k >= 0; --k) {
      double v = f[k];
      for (int l = k + 1; l < r; ++l) v = fma(-Wb[(size_t)l * Nx + k], c[l], v);
      c[k] = bad ? 0.0 : v / alpha[k];
    }
  }
  for (int q = t; q < Nx * r; q += 256) {
    const int a = q / Nx, j = q - a * Nx;
    double s = 0.0;
    for (int b = 0; b < r; ++b) s = fma(B[(size_t)b * Nx + j], M[(size_t)a * r + b], s);
    BM[q] = s;
  }
}

// ---------------------------------------------------------------------------
// The predicted field tables of every parameter (eq.
// DMD_approx_potential_subset at t_{tau-1} and t_{tau-1} + dt/2): c_i =
// sum_k beta_ik c_k, Phi0 = B c_i, Phih = (B M) c_i, and the cell fields
// e_j = (Phi_{j+1} - Phi_j) / h_i into e0, eh (p x N_x row-major).  One
// block per parameter.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) dmd_tables_kernel(const double* __restrict__ B,
                                                         const double* __restrict__ BM,
                                                         const double* __restrict__ C,
                                                         const double* __restrict__ beta,
                                                         const int* __restrict__ rin, int Nx,
                                                         int pstar, const double* __restrict__ h,
                                                         double* __restrict__ e0,
                                                         double* __restrict__ eh) {
  __shared__ double ci[64];
  __shared__ double ph0[SYMROM_MAX_NX], phh[SYMROM_MAX_NX];
  const int i = blockIdx.x;
  const int r = rin[0];
  const int t = threadIdx.x;
  if (t < r) {
    double s = 0.0;
    for (int k = 0; k < pstar; ++k) s = fma(beta[(size_t)i * pstar + k], C[(size_t)k * r + t], s);
    ci[t] = s;
  }
  __syncthreads();
  for (int j = t; j < Nx; j += blockDim.x) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < r; ++q) {
      a = fma(B[(size_t)q * Nx + j], ci[q], a);
      b = fma(BM[(size_t)q * Nx + j], ci[q], b);
    }
    ph0[j] = a;
    phh[j] = b;
  }
  __syncthreads();
  const double hi = h[i];
  for (int j = t; j < Nx; j += blockDim.x) {
    const int jn = (j + 1 == Nx) ? 0 : j + 1;
    e0[(size_t)i * Nx + j] = (ph0[jn] - ph0[j]) / hi;
    eh[(size_t)i * Nx + j] = (phh[jn] - phh[j]) / hi;
  }
}

// ---------------------------------------------------------------------------
// The fixed point of the coefficients with the DMD-DEIM gradient (eq.
// grHDD), whole, one column per block (64 lanes): the predicted potential
// does not depend on Z, so a column needs only its own d sampled rows.
//   k1 = -i g^DD(U0, Z0; e0)   (start value),
//   repeat: Ze = Z0 + dt/2 k;  k' = -i g^DD(U_half, Ze; eh);  stop when
//   |k' - k| / |k'| < tol, or by the stagnation rule (the smaller of the last
//   two updates below stall_tol and the update not decreasing), or after
//   max_iters (the column stays active: ENOCONV); with fixed > 0 exactly
//   that many iterations and no test.
// g^DD = g_F + (C1 Z - conj(C2) conj(Z)) / 2 with g_F[k] = sum_r
// conj(U~[I_r, k]) w_r (q/m) e[j(x_r)], C1 = U~^* U~, C2 = U~^T U~ (the
// arithmetic of the DEIM gather and of the fused fixed-point update).
// Out: k, ZG (the last evaluation point), prev (last relative update),
// active, counters [0] columns left, [1] stalled, [2] largest iteration
// count, [6..7] largest stall-accepted update.
// ---------------------------------------------------------------------------
constexpr int DMD_FP_NC = 30;  // n <= 30 (2n <= 60)

__global__ void __launch_bounds__(64) dmd_fp_kernel(DmdFpArgs a) {
  __shared__ cplx Ud[64 * DMD_FP_NC];
  __shared__ cplx Cs[2 * DMD_FP_NC * DMD_FP_NC];
  __shared__ cplx ze[DMD_FP_NC];
  __shared__ double Fw[64];
  __shared__ double buf[128];
  __shared__ int done_s;
  const int i = blockIdx.x;
  const int L = threadIdx.x;
  const int n = a.n, d = a.d, Nx = a.Nx;
  const double fac = a.factor[i];
  const double wl = (L < d) ? a.w[L] : 0.0;
  cplx z0v = mk(0.0, 0.0), kcur = mk(0.0, 0.0);
  if (L < n) z0v = a.Z0[(size_t)i * n + L];
  // one evaluation of k = -i g^DD at the point in ze with the rows in Ud,
  // the linear part from C (2 n^2) and the field table e (this column)
  auto eval = [&](const double* __restrict__ e) -> cplx {
    if (L < d) {
      double x = 0.0;
      for (int k = 0; k < n; ++k) {
        const cplx u = Ud[L * n + k];
        x = fma(u.re, ze[k].re, x);
        x = fma(-u.im, ze[k].im, x);
      }
      int j;
      double th;
      cell_of(x, fac, Nx, j, th);
      Fw[L] = wl * a.qm * e[(size_t)i * Nx + j];
    }
    __syncthreads();
    cplx knew = mk(0.0, 0.0);
    if (L < n) {
      cplx sk = mk(0.0, 0.0);
      for (int r = 0; r < d; ++r) {
        const cplx u = Ud[r * n + L];
        sk.re = fma(u.re, Fw[r], sk.re);
        sk.im = fma(-u.im, Fw[r], sk.im);
      }
      cplx sl = mk(0.0, 0.0);
      for (int b = 0; b < n; ++b) {
        cfma(sl, Cs[b * n + L], ze[b]);
        cfma(sl, cscale(cconj(Cs[n * n + b * n + L]), -1.0), cconj(ze[b]));
      }
      const cplx g = cadd(sk, cscale(sl, 0.5));
      knew = mk(g.im, -g.re);
    }
    __syncthreads();
    return knew;
  };
  // start value at (U0, Z0) with the table at t_{tau-1}
  if (L < d)
    for (int k = 0; k < n; ++k) Ud[L * n + k] = a.U0[(size_t)k * a.N + a.idx[L]];
  for (int q = L; q < 2 * n * n; q += 64) Cs[q] = a.C12a[q];
  if (L < n) ze[L] = z0v;
  __syncthreads();
  kcur = eval(a.e0);
  // the iterations at U_half with the table at t_{tau-1} + dt/2
  if (L < d)
    for (int k = 0; k < n; ++k) Ud[L * n + k] = a.Uh[(size_t)k * a.N + a.idx[L]];
  for (int q = L; q < 2 * n * n; q += 64) Cs[q] = a.C12[q];
  double prev = INFINITY, rel = 0.0;
  int its = 0;
  bool done = false;
  const int limit = a.fixed > 0 ? a.fixed : a.max_iters;
  while (its < limit) {
    ++its;
    if (L < n) ze[L] = mk(z0v.re + 0.5 * a.dt * kcur.re, z0v.im + 0.5 * a.dt * kcur.im);
    __syncthreads();
    const cplx knew = eval(a.eh);
    if (L < n) {
      const cplx dk = csub(knew, kcur);
      buf[L] = cabs2(dk);
      buf[64 + L] = cabs2(knew);
      a.ZG[(size_t)i * n + L] = ze[L];
    }
    __syncthreads();
    if (L == 0) {
      double dn = 0.0, kn = 0.0;
      for (int q = 0; q < n; ++q) {
        dn += buf[q];
        kn += buf[64 + q];
      }
      bool fin = false;
      if (a.fixed == 0) {
        rel = (kn > 0.0) ? sqrt(dn) / sqrt(kn) : sqrt(dn);
        const bool conv = rel < a.tol;
        const bool stall = !conv && rel >= prev && fmin(rel, prev) < a.stall_tol;
        prev = rel;
        fin = conv || stall;
        if (stall) {
          atomicAdd(&a.counters[1], 1);
          atomicMax(reinterpret_cast<unsigned long long*>(a.counters + 6),
                    (unsigned long long)__double_as_longlong(rel));
        }
      }
      done_s = fin ? 1 : 0;
    }
    kcur = knew;
    __syncthreads();
    done = done_s != 0;
    if (done) break;
  }
  if (L < n) a.k[(size_t)i * n + L] = kcur;
  if (L == 0) {
    const bool left = a.fixed == 0 && !done;
    a.prev[i] = prev;
    a.active[i] = left ? 1 : 0;
    if (left) atomicAdd(&a.counters[0], 1);
    atomicMax(&a.counters[2], its);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_subset_select(hipStream_t s, const cplx* Z, int n, int p, int pstar, double* dmin,
                          int* S) {
  hipLaunchKernelGGL(subset_select_kernel, dim3(1), dim3(256), 0, s, Z, n, p, pstar, dmin, S);
}

void launch_rbf_weights(hipStream_t s, const double* eta, int dim, int p, const int* S, int pstar,
                        int* member, double* beta, int* flags) {
  hipLaunchKernelGGL(rbf_weights_kernel, dim3(1), dim3(256), 0, s, eta, dim, p, S, pstar, member,
                     beta, flags);
}

void launch_grid_rows(hipStream_t s, const double* src, const int* cols, int k, int Nx,
                      double* dst) {
  hipLaunchKernelGGL(grid_rows_kernel, dim3(k), dim3(256), 0, s, src, cols, k, Nx, dst);
}

void launch_gather_zcols(hipStream_t s, const cplx* Z, int n, const int* S, int k, cplx* out) {
  const int tot = n * k;
  hipLaunchKernelGGL(gather_zcols_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, Z, n, S, k,
                     out);
}

void launch_dmd_operator(hipStream_t s, const DmdChainArgs& c) {
  const int P = c.pstar * c.T;
  hipLaunchKernelGGL(dmd_window_kernel, dim3(P), dim3(256), 0, s, c.ring, c.nslots, c.base,
                     c.pstar, c.T, c.Nx, c.Y, c.Yp);
  // the QR works on a copy of Y (its reflectors stay there)
  (void)hipMemcpyAsync(c.W, c.Y, (size_t)c.Nx * P * sizeof(double), hipMemcpyDeviceToDevice, s);
  ALLOW_BIG_LDS(dmd_svd_kernel);
  hipLaunchKernelGGL(dmd_svd_kernel, dim3(1), dim3(256), (2 * 64 * 65 + 8192) * sizeof(double), s, c.W,
                     c.Nx, P, c.tol, c.sig, c.V, c.rdev, c.U, c.flags);
  hipLaunchKernelGGL(dmd_form_kernel, dim3(1), dim3(256), 0, s, c.Yp, c.Nx, P, c.sig, c.V,
                     c.rdev, c.B, c.U, c.A);
  const size_t lds = (size_t)4 * DMD_MAX_R * DMD_MAX_R * sizeof(cplx);
  ALLOW_BIG_LDS(dmd_eig_kernel);
  hipLaunchKernelGGL(dmd_eig_kernel, dim3(1), dim3(64), lds, s, c.A, c.rdev, c.M, c.lam, c.flags);
  // the last window level of the subset, as the right-hand sides of B^+
  hipLaunchKernelGGL(grid_rows_kernel, dim3(c.pstar), dim3(256), 0, s,
                     c.ring + (size_t)((c.base + c.T) % c.nslots) * c.pstar * c.Nx, nullptr,
                     c.pstar, c.Nx, c.Wf);
  hipLaunchKernelGGL(dmd_coords_kernel, dim3(1), dim3(256), 0, s, c.B, c.M, c.rdev, c.Nx,
                     c.pstar, c.Wb, c.Wf, c.C, c.BM, c.flags);
}

void launch_dmd_tables(hipStream_t s, const DmdChainArgs& c, int p, const double* beta,
                       const double* h, double* e0, double* eh) {
  hipLaunchKernelGGL(dmd_tables_kernel, dim3(p), dim3(256), 0, s, c.B, c.BM, c.C, beta, c.rdev,
                     c.Nx, c.pstar, h, e0, eh);
}

void launch_dmd_fp(hipStream_t s, const DmdFpArgs& a, int p) {
  hipLaunchKernelGGL(dmd_fp_kernel, dim3(p), dim3(64), 0, s, a);
}
