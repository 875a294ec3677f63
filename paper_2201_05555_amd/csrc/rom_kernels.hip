// Streaming kernels of the reduced model: field gather at reconstructed
// particles, tall-skinny products with reduction over particles (split over
// row blocks, reduced in a fixed order), and row-wise small products.
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
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

// Reconstruct X = Re(U~ Z~), V = Im(U~ Z~) (nout x p each): every row
// (rows == nullptr, nout = N) or the rows listed in rows[0 .. nout) (a row
// index outside [0, N) gives NaN in its output row).
template <int NC>
__global__ void __launch_bounds__(256) reconstruct_kernel(const cplx* __restrict__ U, int N, int n,
                                                          const cplx* __restrict__ Z, int p,
                                                          double* __restrict__ X,
                                                          double* __restrict__ V,
                                                          const int* __restrict__ rows, int nout) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nout) return;
  const int src = rows ? rows[l] : l;
  const bool in = src >= 0 && src < N;
  const int sc = in ? src : 0;
  cplx u[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) u[k] = (k < n) ? U[(size_t)k * N + sc] : mk(0.0, 0.0);
  for (int i = 0; i < p; ++i) {
    cplx acc = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < NC; ++k)
      if (k < n) cfma(acc, u[k], Z[(size_t)i * n + k]);
    if (!in) acc = mk(NAN, NAN);
    if (X) X[(size_t)i * nout + l] = acc.re;
    if (V) V[(size_t)i * nout + l] = acc.im;
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
  // eight partials of a lane in flight at once (clamped loads, masked adds)
  for (int k0 = lane; k0 < nkb; k0 += 8 * 64) {
    cplx v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)min(k0 + 64 * u, nkb - 1) * nout + o];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = k0 + 64 * u < nkb;
      re += in ? v[u].re : 0.0;
      im += in ? v[u].im : 0.0;
    }
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
__global__ void __launch_bounds__(256) rowgemm_kernel(RowTerms T, int N, int m, cplx* out,
                                                      int accum) {
  extern __shared__ cplx Ms[];
  int off = 0;
  for (int s = 0; s < T.count; ++s) {
    // M_s is k_s x m with leading dimension ld_s (k_s when ld_s is 0)
    const int ks = T.k[s], ld = T.ld[s] ? T.ld[s] : ks;
    for (int t = threadIdx.x; t < ks * m; t += blockDim.x)
      Ms[off + t] = T.M[s][(size_t)(t / ks) * ld + t % ks];
    off += ks * m;
  }
  __syncthreads();
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= N) return;
  cplx acc[MC];
#pragma unroll
  for (int o = 0; o < MC; ++o) acc[o] = (accum && o < m) ? out[(size_t)o * N + l] : mk(0.0, 0.0);
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

// The row combination for m <= 8 output columns that also forms the split-K
// partials of the Gram of [P, O] (P: kp <= 8 optional leading columns read
// from `pre`, O the output): the block's rows are kept in LDS and each
// upper-triangle entry (i <= j) is summed over four 64-row chunks, the
// chunks then in order; part[block][j g + i] holds the entry and
// part[block][i g + j] its conjugate, g = kp + m (the layout of
// gemm_ah_b_kernel).
template <int MC, bool PRE>
__global__ void __launch_bounds__(256) rowgemm_gram_kernel(RowTerms T, int N, int m,
                                                           cplx* __restrict__ out,
                                                           const cplx* __restrict__ pre, int kp,
                                                           cplx* __restrict__ part) {
  constexpr int GW = PRE ? 2 * MC : MC;  // LDS row width
  extern __shared__ cplx Ms[];
  __shared__ cplx Os[256 * GW];
  __shared__ cplx red[4][GW * (GW + 1) / 2];
  int off = 0;
  for (int s = 0; s < T.count; ++s) {
    for (int t = threadIdx.x; t < T.k[s] * m; t += blockDim.x) Ms[off + t] = T.M[s][t];
    off += T.k[s] * m;
  }
  __syncthreads();
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int kpp = PRE ? kp : 0;
  cplx acc[MC];
#pragma unroll
  for (int o = 0; o < MC; ++o) acc[o] = mk(0.0, 0.0);
  if (l < N) {
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
  // rows past N stay zero and add nothing
  cplx* orow = Os + threadIdx.x * GW;
  if (PRE)
    for (int k = 0; k < kpp; ++k) orow[k] = (l < N) ? pre[(size_t)k * N + l] : mk(0.0, 0.0);
#pragma unroll
  for (int o = 0; o < MC; ++o)
    if (o < m) orow[kpp + o] = acc[o];
  __syncthreads();
  const int g = kpp + m;
  const int npair = g * (g + 1) / 2;
  for (int it = threadIdx.x; it < 4 * npair; it += blockDim.x) {
    const int chunk = it / npair, pr = it - chunk * npair;
    // pair index -> (i, j), i <= j, column by column
    int q = pr, pj = 0;
    while (q > pj) {
      q -= pj + 1;
      ++pj;
    }
    const int pi = q;
    cplx sacc = mk(0.0, 0.0);
    for (int rr = 0; rr < 64; ++rr) {
      const cplx* row = Os + (chunk * 64 + rr) * GW;
      cfma(sacc, cconj(row[pi]), row[pj]);
    }
    red[chunk][pr] = sacc;
  }
  __syncthreads();
  for (int pr = threadIdx.x; pr < npair; pr += blockDim.x) {
    int q = pr, pj = 0;
    while (q > pj) {
      q -= pj + 1;
      ++pj;
    }
    const int pi = q;
    cplx gs = red[0][pr];
    for (int c = 1; c < 4; ++c) gs = cadd(gs, red[c][pr]);
    cplx* pb = part + (size_t)blockIdx.x * g * g;
    pb[pj * g + pi] = gs;
    if (pi != pj) pb[pi * g + pj] = cconj(gs);
  }
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
    const int* __restrict__ active, cplx* __restrict__ gF, const int* __restrict__ gate,
    DeimStartArgs st) {
  if (gate && gate[0] == 0) return;
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
    if (st.k) {
      // k = -i (gF + (C1 Z - conj(C2) conj(Z)) / 2) for this entry (the DEIM
      // reduced gradient with its linear part i U~^* V_r, C1 = U~^* U~,
      // C2 = U~^T U~), then the first iterate Z0 + h k (the arithmetic of
      // dense_finish_z_kernel)
      cplx sl = mk(0.0, 0.0);
      for (int b = 0; b < n; ++b) {
        cfma(sl, st.C12[b * n + k], zi[b]);
        cfma(sl, cscale(cconj(st.C12[n * n + b * n + k]), -1.0), cconj(zi[b]));
      }
      const cplx g = cadd(s, cscale(sl, 0.5));
      const cplx kk = mk(g.im, -g.re);
      const size_t t = (size_t)i * n + k;
      st.k[t] = kk;
      st.Zev[t] = mk(zi[k].re + st.h * kk.re, zi[k].im + st.h * kk.im);
    }
  }
  if (st.k) {
    // start of the fixed point (as fp_init_kernel): column i active, no
    // previous update; block 0 resets the counters
    if (threadIdx.x == 0) {
      st.prev[i] = INFINITY;
      st.active[i] = 1;
    }
    if (i == 0 && threadIdx.x < 4) st.counters[threadIdx.x] = (threadIdx.x == 0) ? p : 0;
    if (i == 0 && (threadIdx.x == 6 || threadIdx.x == 7)) st.counters[threadIdx.x] = 0;
  }
}


// ---------------------------------------------------------------------------
// Fused gather + projection (eq. grads) on the FP64 matrix cores: the field
// part U~^* F of g = U~^* G~, G~ = F + i v, with F = (q/m) e_c at the
// particle's cell evaluated on the fly and never stored (the velocity part
// i U~^* v, v = Im(U~ Z~), is linear in Z~ and is added by the reduction
// from the small Gram matrices of U~).  A block takes a tile of 16 CBN
// parameters (their field rows in LDS with ET_LDS) and a range of particle
// rows, each of its WV wavefronts 16 rows at a time.  Real form with K = 2
// NC: a = [Re U~ | -Im U~] (row-major per particle), b = [Re Z~; Im Z~], so
// that the positions X = a b (16 rows x 16 parameters per accumulator, CBN
// accumulators).  In the accumulator layout lane l holds X[4 v + l / 16][l %
// 16], which is the layout of the B operand of g = a^T F for the 4-row step
// v: the cell, the field lookup and the masks run on the positions in
// registers and feed the second product directly.  Results: row block b
// writes part[b * rec + c * n + k] and, with want_colsq, |F[:, c]|^2 at
// part[b * rec + n * p + c].re; the wavefronts are summed in a fixed order.
// ---------------------------------------------------------------------------
template <int NC, int CBN, bool ET_LDS, int WV>
__global__ void __launch_bounds__(64 * WV) gather_project_mfma_kernel(
    const cplx* __restrict__ U, int N, int n, const cplx* __restrict__ Z, int p, int Nx, int rpb,
    const double* __restrict__ factor, const double* __restrict__ e, double qm,
    const int* __restrict__ active, int rec, int want_colsq, cplx* __restrict__ part,
    const int* __restrict__ gate) {
  if (gate && gate[0] == 0) return;
  constexpr int KS = (2 * NC + 3) / 4;    // 4-deep steps of the position product
  constexpr int MT = (2 * NC + 15) / 16;  // 16-row tiles of the projection
  constexpr int PT = 16 * CBN;            // parameters of the tile
  extern __shared__ double smem[];
  double* et = smem;  // [PT][Nx] (ET_LDS); after the rows, the wavefront sums
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  // parameter tiles vary fastest over the grid: blocks of the same rows run
  // together and share the rows of U~ in L2
  const int c0 = blockIdx.x * PT;
  const int ntc = min(PT, p - c0);
  const int rb = blockIdx.y;
  if (ET_LDS) {
    const double* es = e + (size_t)c0 * Nx;
    const int tot = ntc * Nx;
    for (int t0 = 0; t0 < tot; t0 += 4 * 64 * WV) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + u * 64 * WV + tid;
        v[u] = (t < tot) ? es[t] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + u * 64 * WV + tid;
        if (t < tot) et[t] = qm * v[u];
      }
    }
  }
  // B operands of the positions (b[q][parameter 16 cb + li] for q = 4 ks +
  // lk), the factor and the mask of this lane's parameter in each block
  double bz[CBN][KS], fac[CBN];
  bool on[CBN];
#pragma unroll
  for (int cb = 0; cb < CBN; ++cb) {
    const int cl = 16 * cb + li;
    const int c = c0 + min(cl, ntc - 1);
    on[cb] = cl < ntc && (!active || active[c]);
    fac[cb] = factor[c];
    pos_coefs<KS>(Z, n, NC, c, on[cb], lk, bz[cb]);
  }
  mf4 acc[MT][CBN];
  double csq[CBN];
#pragma unroll
  for (int cb = 0; cb < CBN; ++cb) {
    csq[cb] = 0.0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt][cb] = mf4{0.0, 0.0, 0.0, 0.0};
  }
  __syncthreads();
  const int r0 = rb * rpb;
  const int r1 = min(N, r0 + rpb);
  // the operands of U~ for a tile of 16 rows: a[row t0 + li][q = 4 ks + lk]
  // for the positions and a^T[o = 16 mt + li][row t0 + 4 s + lk] for the
  // projection; those of the next tile are loaded while this one computes
  // (the rows stream from memory: each tile would otherwise wait for them)
  // (each operand entry is sgn * a component of U~[col][row], with the
  // column, component and sign fixed per lane: set up once)
  PosRows<KS> pr;
  pr.setup(U, N, n, NC, lk);
  const double* pt_[MT];
  double st_[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int o = 16 * mt + li;
    const int col = (o < NC) ? o : o - NC;
    const bool ok = o < 2 * NC && col < n;
    pt_[mt] = reinterpret_cast<const double*>(U + (size_t)(ok ? col : 0) * N) + (o < NC ? 0 : 1);
    st_[mt] = ok ? (o < NC ? 1.0 : -1.0) : 0.0;
  }
  double a[KS], at[MT][4], an[KS], atn[MT][4];
  auto load_tile = [&](int tt, double* ra, double (*rat)[4]) {
    pr.load(min(tt + li, r1 - 1), ra);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int rw = min(tt + 4 * s4 + lk, r1 - 1);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) rat[mt][s4] = st_[mt] * pt_[mt][2 * (size_t)rw];
    }
  };
  load_tile(r0 + 16 * w, a, at);
  for (int t0 = r0 + 16 * w; t0 < r1; t0 += 16 * WV) {
    load_tile(t0 + 16 * WV, an, atn);
    mf4 X[CBN];
#pragma unroll
    for (int cb = 0; cb < CBN; ++cb) X[cb] = pos_tile<KS>(a, bz[cb]);
    // F at the positions: lane holds row t0 + 4 v + lk, parameter 16 cb + li.
    // All cells first, then all lookups (unconditional: the cell is always
    // in range), then the masks as selects, so that the lookups of a lane
    // are in flight together
    double F[CBN][4];
#pragma unroll
    for (int cb = 0; cb < CBN; ++cb) {
      int jv[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double th;
        cell_of(X[cb][v], fac[cb], Nx, jv[v], th);
      }
      const int cl = min(16 * cb + li, ntc - 1);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        F[cb][v] = ET_LDS ? et[cl * Nx + jv[v]] : qm * e[(size_t)(c0 + cl) * Nx + jv[v]];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        F[cb][v] = (on[cb] && t0 + 4 * v + lk < r1) ? F[cb][v] : 0.0;
        csq[cb] = fma(F[cb][v], F[cb][v], csq[cb]);
      }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int cb = 0; cb < CBN; ++cb)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
          acc[mt][cb] = mfma_f64_step(at[mt][s4], F[cb][s4], acc[mt][cb]);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a[ks] = an[ks];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) at[mt][s4] = atn[mt][s4];
  }
  // the column sums of |F|^2 over the four row groups of a lane's parameter
#pragma unroll
  for (int cb = 0; cb < CBN; ++cb) {
    csq[cb] += __shfl_xor(csq[cb], 16, 64);
    csq[cb] += __shfl_xor(csq[cb], 32, 64);
  }
  __syncthreads();  // (the field rows are no longer needed)
  // wavefront sums: red[w][o][parameter], o over the 16 MT real outputs
  double* red = smem;                          // [WV][16 MT][PT]
  double* rcs = smem + WV * 16 * MT * PT;       // [WV][PT]
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int cb = 0; cb < CBN; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        red[((size_t)w * 16 * MT + 16 * mt + 4 * v + lk) * PT + 16 * cb + li] = acc[mt][cb][v];
  if (lk == 0)
#pragma unroll
    for (int cb = 0; cb < CBN; ++cb) rcs[w * PT + 16 * cb + li] = csq[cb];
  __syncthreads();
  cplx* pb = part + (size_t)rb * rec;
  for (int t = tid; t < ntc * n; t += 64 * WV) {
    const int q = t / n, k = t % n;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int ww = 0; ww < WV; ++ww) {
      re += red[((size_t)ww * 16 * MT + k) * PT + q];
      im += red[((size_t)ww * 16 * MT + NC + k) * PT + q];
    }
    pb[(size_t)(c0 + q) * n + k] = mk(re, im);
  }
  if (want_colsq)
    for (int t = tid; t < ntc; t += 64 * WV) {
      double sw = rcs[t];
#pragma unroll
      for (int ww = 1; ww < WV; ++ww) sw += rcs[ww * PT + t];
      pb[(size_t)n * p + c0 + t] = mk(sw, 0.0);
    }
}

// C1[o] = sum_b part[b][o] for o < n1, C2[o - n1] = the real part of that sum
// for n1 <= o < nout; blocks summed in a fixed order (one wavefront per output).
// With G12 = [U~^* U~, U~^T U~] (n x n each, column-major) and the
// coefficients Z (n x p) given, the velocity part of the gradient is added:
// for o = c n + a < n1, (G1 z - conj(G2 z))_a / 2 with z = Z[:, c] (this is
// i U~^* Im(U~ z)), and for o = n1 + c, |Im(U~ z)|^2 =
// (z^* G1 z - Re(z^T G2 z)) / 2.
__global__ void __launch_bounds__(256) reduce_partials2_kernel(const cplx* __restrict__ part,
                                                               int nkb, int rec, int n1, int nout,
                                                               cplx* __restrict__ C1,
                                                               double* __restrict__ C2,
                                                               const int* __restrict__ gate,
                                                               const cplx* __restrict__ G12,
                                                               const cplx* __restrict__ Z, int n) {
  if (gate && gate[0] == 0) return;
  const int lane = threadIdx.x & 63;
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (o >= nout) return;
  double re = 0.0, im = 0.0;
  // eight partials of a lane in flight at once (clamped loads, masked adds)
  for (int k0 = lane; k0 < nkb; k0 += 8 * 64) {
    cplx v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)min(k0 + 64 * u, nkb - 1) * rec + o];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = k0 + 64 * u < nkb;
      re += in ? v[u].re : 0.0;
      im += in ? v[u].im : 0.0;
    }
  }
  if (G12) {
    const cplx* G1 = G12;
    const cplx* G2 = G12 + (size_t)n * n;
    if (o < n1) {
      const int c = o / n, a = o - c * n;
      const cplx* z = Z + (size_t)c * n;
      for (int b = lane; b < n; b += 64) {
        cplx t1 = mk(0.0, 0.0), t2 = mk(0.0, 0.0);
        cfma(t1, G1[(size_t)b * n + a], z[b]);
        cfma(t2, G2[(size_t)b * n + a], z[b]);
        re += 0.5 * (t1.re - t2.re);
        im += 0.5 * (t1.im + t2.im);
      }
    } else {
      const int c = o - n1;
      const cplx* z = Z + (size_t)c * n;
      for (int t = lane; t < n * n; t += 64) {
        const int b = t / n, a = t - b * n;
        cplx t1 = mk(0.0, 0.0), t2 = mk(0.0, 0.0);
        cfma(t1, G1[(size_t)b * n + a], z[b]);  // G1[a][b] z_b
        cfma(t2, G2[(size_t)b * n + a], z[b]);  // G2[a][b] z_b
        const cplx za = z[a];
        // Re(conj(z_a) t1) - Re(z_a t2)
        re += 0.5 * ((za.re * t1.re + za.im * t1.im) - (za.re * t2.re - za.im * t2.im));
      }
    }
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
// with G~ = F + i v.  Only the field part F (-i h Q) is evaluated per
// particle and parameter (F at the particle's cell, never stored); the
// velocity part h v Q, v = Im(U~ Z~), equals U~ (-(i h / 2) Z~ Q) +
// conj(U~) ((i h / 2) conj(Z~) Q), two n x n products per row.  Q (p x n,
// ld p) and MU (n x n, ld n) as written by the dense kernels; with g (n x p,
// the projection g~) given instead of MU, every block forms MU = i h g~^T Q
// itself, and every block forms M = MU - (i h / 2) Z~ Q and N = (i h / 2)
// conj(Z~) Q (eight lanes per entry).  The products run on the FP64 matrix
// cores.  Each wavefront takes 64 particle rows (four 16-row tiles)
// and walks the parameters 16 at a time: the positions come from pos_tile
// (the code of the deposit and the gather-projection, so the cells agree),
// an LDS transpose gives each lane one row and the 16 parameters (the
// lookups of a wavefront then fall in one parameter's field row), a second
// one gives the A operand of aq = F (-i h Q) in real form (outputs o: the
// real parts of the n columns, then the imaginary parts), accumulated on
// the matrix cores.  At the end the outputs of a row are gathered through
// LDS and U~ M + conj(U~) N is added per row.
// ---------------------------------------------------------------------------
template <int NC>
__global__ void __launch_bounds__(256) gather_xi_mfma_kernel(
    const cplx* __restrict__ U, int N, int n, const cplx* __restrict__ Z, int p, int Nx,
    const double* __restrict__ factor, const double* __restrict__ e, double qm,
    const cplx* __restrict__ Q, const cplx* __restrict__ MU, const cplx* __restrict__ gp,
    double h, cplx* __restrict__ out) {
  constexpr int KS = (2 * NC + 3) / 4;
  constexpr int MT = (2 * NC + 15) / 16;
  constexpr int XS = 65;  // row stride of the position tile (parameter-major)
  constexpr int FS = 17;  // row stride of the field tile (row-major)
  constexpr int OS = 16 * MT + 1;  // row stride of the output tile (>= FS)
  // one region per wavefront holds the position tile, then the field tile,
  // then the output tile (each read whole before the next is written)
  constexpr int WS = (16 * XS > 64 * OS) ? 16 * XS : 64 * OS;
  __shared__ cplx Ms[NC * NC], Ns[NC * NC];
  __shared__ double Ws[4][WS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  {
    // M = MU - (i h / 2) Z~ Q (MU = i h g~ Q formed here when g is given),
    // N = (i h / 2) conj(Z~) Q; lanes 8e..8e+7 split the sums over c
    const int e8 = tid >> 3, part8 = tid & 7;
    for (int e0 = 0; e0 < NC * NC; e0 += 32) {
      const int t = e0 + e8;
      const int j = t / NC, k = t % NC;
      cplx sm = mk(0.0, 0.0), sn = mk(0.0, 0.0);
      if (t < NC * NC && j < n && k < n) {
        for (int c0 = part8; c0 < p; c0 += 64) {
          cplx gv[8], zv[8], qv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int c = min(c0 + 8 * u, p - 1);
            gv[u] = gp ? gp[(size_t)c * n + j] : mk(0.0, 0.0);
            zv[u] = Z[(size_t)c * n + j];
            qv[u] = Q[(size_t)k * p + c];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (c0 + 8 * u < p) {
              const cplx mq = mk(h * qv[u].im, -h * qv[u].re);
              cfma(sm, mk(gv[u].re - 0.5 * zv[u].re, gv[u].im - 0.5 * zv[u].im), mq);
              cfmac(sn, zv[u], mq);
            }
        }
      }
#pragma unroll
      for (int o = 4; o >= 1; o >>= 1) {
        sm.re += __shfl_xor(sm.re, o, 64);
        sm.im += __shfl_xor(sm.im, o, 64);
        sn.re += __shfl_xor(sn.re, o, 64);
        sn.im += __shfl_xor(sn.im, o, 64);
      }
      if (part8 == 0 && t < NC * NC) {
        const bool in = j < n && k < n;
        const cplx mu = (in && !gp) ? MU[(size_t)k * n + j] : mk(0.0, 0.0);
        Ms[t] = in ? mk(mu.re - sm.re, mu.im - sm.im) : mk(0.0, 0.0);
        Ns[t] = in ? mk(-0.5 * sn.re, -0.5 * sn.im) : mk(0.0, 0.0);
      }
    }
  }
  __syncthreads();
  const int rbase = (blockIdx.x * 4 + w) * 64;  // this wavefront's 64 rows
  if (rbase >= N) return;
  const int rlast = N - 1;
  PosRows<KS> pr;
  pr.setup(U, N, n, NC, lk);
  double a[4][KS];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) pr.load(min(rbase + 16 * rt + li, rlast), a[rt]);
  mf4 acc[4][MT];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[rt][mt] = mf4{0.0, 0.0, 0.0, 0.0};
  double* xs = Ws[w];
  double* fs = Ws[w];
  for (int c0 = 0; c0 < p; c0 += 16) {
    const int ntc = min(16, p - c0);
    // B operands: the coefficients of parameter c0 + li and the entries
    // qr[c0 + 4 s + lk][o = 16 mt + li] of -i h Q in real form
    double bz[KS];
    pos_coefs<KS>(Z, n, NC, c0 + min(li, ntc - 1), li < ntc, lk, bz);
    double qb[MT][4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int c = c0 + 4 * s4 + lk;
      const bool cv = 4 * s4 + lk < ntc;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int o = 16 * mt + li;
        const int k = (o < NC) ? o : o - NC;
        const bool ok = cv && o < 2 * NC && k < n;
        const cplx qv = Q[(size_t)(ok ? k : 0) * p + min(c, p - 1)];
        // -i h q = (h q.im, -h q.re)
        qb[mt][s4] = ok ? ((o < NC) ? h * qv.im : -h * qv.re) : 0.0;
      }
    }
    // positions, parameter-major in LDS: xs[param li][row 16 rt + 4 v + lk]
    // (after the last tile's field reads)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const mf4 X = pos_tile<KS>(a[rt], bz);
#pragma unroll
      for (int v = 0; v < 4; ++v) xs[li * XS + 16 * rt + 4 * v + lk] = X[v];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // lane = row rbase + lane: its 16 positions, cells and field values
    // (parameter q uniform across the wavefront: one field row per lookup;
    // all 16 lookups in flight together)
    {
      int jq[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        double th;
        cell_of(xs[q * XS + lane], factor[c0 + min(q, ntc - 1)], Nx, jq[q], th);
      }
      double fq[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) fq[q] = e[(size_t)(c0 + min(q, ntc - 1)) * Nx + jq[q]];
      // (the positions are read: the field tile takes their place)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int q = 0; q < 16; ++q) fs[lane * FS + q] = (q < ntc) ? qm * fq[q] : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // aq += F qr: A[row 16 rt + li][parameter 4 s + lk] from the field tile
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const double fa = fs[(16 * rt + li) * FS + 4 * s4 + lk];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[rt][mt] = mfma_f64_step(fa, qb[mt][s4], acc[rt][mt]);
      }
  }
  // the outputs of each row through LDS (the field tile's space): lane holds
  // aq[row 16 rt + 4 v + lk][o = 16 mt + li]
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double* os = fs;  // [64][OS]
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) os[(16 * rt + 4 * v + lk) * OS + 16 * mt + li] = acc[rt][mt][v];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int l = rbase + lane;
  if (l < N) {
    cplx u[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) u[k] = (k < n) ? U[(size_t)k * N + l] : mk(0.0, 0.0);
    // out[:, k] = aq[k] + (U~ M + conj(U~) N)[:, k], one column at a time
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      cplx r = mk(os[lane * OS + k], os[lane * OS + NC + k]);
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        cfma(r, u[j], Ms[j * NC + k]);
        cfmac(r, u[j], Ns[j * NC + k]);
      }
      if (k < n) out[(size_t)k * N + l] = r;
      asm volatile("" ::: "memory");
    }
  }
}

// ---------------------------------------------------------------------------
// DEIM basis, indices and weights (Sec. 4.2.2), N-wide passes.
// ---------------------------------------------------------------------------

// (value, index) pairs: the larger value wins, the smaller index on ties
__device__ __forceinline__ void dg_take(double& best, int& bi, double ov, int oi) {
  if (ov > best || (ov == best && oi < bi)) {
    best = ov;
    bi = oi;
  }
}

// winner over the 64 lanes of a wavefront, the same in every lane: row
// butterflies, then the four row winners in a fixed order
__device__ __forceinline__ void dg_wave_argmax(double& best, int& bi) {
  dg_take(best, bi, bfly64<0>(best), bfly32<0>(bi));
  dg_take(best, bi, bfly64<1>(best), bfly32<1>(bi));
  dg_take(best, bi, bfly64<2>(best), bfly32<2>(bi));
  dg_take(best, bi, bfly64<3>(best), bfly32<3>(bi));
  double rv[4];
  int ri[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    rv[q] = rdlane64(best, 16 * q);
    ri[q] = __builtin_amdgcn_readlane(bi, 16 * q);
  }
  best = rv[0];
  bi = ri[0];
#pragma unroll
  for (int q = 1; q < 4; ++q) dg_take(best, bi, rv[q], ri[q]);
}

// winner of per-block (value, index) results: largest value, smallest index
// on ties; computed by the first wavefront, returned in its lanes
__device__ int dg_winner(const double* __restrict__ val, const int* __restrict__ idx, int nb) {
  const int lane = threadIdx.x & 63;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int b = lane; b < nb; b += 64) dg_take(best, bi, val[b], idx[b]);
  dg_wave_argmax(best, bi);
  return bi;
}

// The index of position pos: the winner of the previous pass, or, with the
// adaptive update (Sec. 4.2.2, eq. indices_adaptive_DEIM), the inherited
// index forced[pos] when it is set and not chosen at an earlier position.
__device__ int dg_choose(const double* __restrict__ pval, const int* __restrict__ pidx, int nprev,
                         const int* __restrict__ forced, const int* __restrict__ idx, int pos,
                         int N) {
  int win = dg_winner(pval, pidx, nprev);
  if (forced) {
    const int f = forced[pos];
    if (f >= 0 && f < N) {
      bool dup = false;
      for (int q = 0; q < pos; ++q) dup |= (idx[q] == f);
      if (!dup) win = f;
    }
  }
  return win;
}

// Greedy DEIM step k (the selection rule of Sec. 4.2.2): l_k = argmax |r_k|,
// r_k = psi_k - Psi_{k-1} c_k, M_k c_k = P^T psi_k with M_k = P^T Psi_{k-1}
// (k x k; rows l_0 .. l_{k-1}).  Instead of a fresh solve per step, the
// inverse of M_k is carried from pass to pass by bordering: with
// B = M_{k-1}^{-1} and u = c_{k-1} from the previous pass, the new row
// b = Psi[l_{k-1}, 0..k-2], delta = Psi[l_{k-1}, k-1] and the Schur complement
// s = delta - b.u (the winning residual itself),
//   M_k^{-1} = [[B + u v^T / s, -u / s], [-v^T / s, 1 / s]],  v = B^T b,
//   c_k = [B y' - tau u ; tau],  tau = (y_last - v.y') / s,
// where y' = Psi[l_0..l_{k-2}, k] and y_last = Psi[l_{k-1}, k].  Every block
// forms c_k redundantly (wavefront 0); block 0 also writes M_k^{-1} and c_k
// for the next pass and records l_{k-1} = the winner of the previous pass
// (pval, pidx: nprev block results).  Each block then writes the (value,
// index) of the largest |r_k| over its rows (smallest index on ties) to bval,
// bidx.  k = 0 takes r_0 = psi_0.  Inverses are kept as 64 x 64 row-major.
#define DG_KR 16   // leading columns of Psi prefetched for a thread's first two rows
__device__ __forceinline__ double dg_wave_sum(double v) { return wave_sum64(v); }

// Bordering step shared by the greedy passes and the weights: reads
// Bprev (m x m, m = k - 1), uprev (m), the rows idx[0..m-1] and l = lwin;
// leaves c_k in cs[0..k-1], v in vs, u in us, B in Bs and s in sh_s.
__device__ void dg_border(const double* __restrict__ Psi, int N, int k, int ycol,
                          const int* __restrict__ idx, int l, double* Bs, double* us,
                          double* ys, double* bs, double* cs, double* vs, double* sh_s) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int m = k - 1;
  if (tid < m) bs[tid] = Psi[(size_t)tid * N + l];
  __syncthreads();
  if (tid < 64) {
    const double delta = Psi[(size_t)m * N + l];
    const double ylast = (ycol >= 0) ? Psi[(size_t)ycol * N + l] : 0.0;
    double vj = 0.0, zj = 0.0;
    for (int i = 0; i < m; ++i) {
      vj = fma(Bs[i * 65 + lane], bs[i], vj);   // (B^T b)_lane
      zj = fma(Bs[lane * 65 + i], ys[i], zj);   // (B y')_lane
    }
    const double ul = us[lane], bl = bs[lane], yl = ys[lane];
    vj = (lane < m) ? vj : 0.0;
    zj = (lane < m) ? zj : 0.0;
    const double s = delta - dg_wave_sum((lane < m) ? bl * ul : 0.0);
    const double vy = dg_wave_sum((lane < m) ? vj * yl : 0.0);
    const double tau = (ylast - vy) / s;
    cs[lane] = (lane < m) ? zj - tau * ul : ((lane == m) ? tau : 0.0);
    vs[lane] = vj;
    if (lane == 0) *sh_s = s;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) deim_greedy_kernel(
    const double* __restrict__ Psi, int N, int k, int* __restrict__ idx,
    const double* __restrict__ pval, const int* __restrict__ pidx, int nprev,
    double* __restrict__ bval, int* __restrict__ bidx, const double* __restrict__ Bprev,
    const double* __restrict__ uprev, double* __restrict__ Bnext, double* __restrict__ cnext,
    int* __restrict__ flags, const int* __restrict__ forced) {
  __shared__ double Bs[64 * 65];
  __shared__ double us[64], ys[64], bs[64], cs[64], vs[64], cf[64];
  __shared__ double sh_s;
  __shared__ double sv[4];
  __shared__ int si[4];
  __shared__ int lwin;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int stride = gridDim.x * 256;
  // the leading entries of this thread's first two rows, loaded before the
  // winner is known (addresses clamped in range; unused entries ignored)
  const int l0 = blockIdx.x * 256 + tid, l1 = l0 + stride;
  const int l0c = min(l0, N - 1), l1c = min(l1, N - 1);
  double p0[DG_KR], p1[DG_KR];
#pragma unroll
  for (int q = 0; q < DG_KR; ++q) {
    const int qc = min(q, k);
    p0[q] = Psi[(size_t)qc * N + l0c];
    p1[q] = Psi[(size_t)qc * N + l1c];
  }
  if (k > 0) {
    const int m = k - 1;
    for (int t = tid; t < m * m; t += 256) {
      const int i = t / m, j = t - i * m;
      Bs[i * 65 + j] = Bprev[i * 64 + j];
    }
    if (tid < 64) {
      us[tid] = (tid < m) ? uprev[tid] : 0.0;
      ys[tid] = (tid < m) ? Psi[(size_t)k * N + idx[tid]] : 0.0;
      bs[tid] = 0.0;
    }
    if (w == 0) {
      int win = dg_choose(pval, pidx, nprev, forced, idx, k - 1, N);
      if (win < 0 || win >= N) {
        // no finite residual anywhere: report, and keep the row in range
        if (lane == 0 && blockIdx.x == 0 && flags) flags[0] |= 16;
        win = 0;
      }
      if (lane == 0) {
        lwin = win;
        if (blockIdx.x == 0) idx[k - 1] = win;
      }
    }
    __syncthreads();
    dg_border(Psi, N, k, k, idx, lwin, Bs, us, ys, bs, cs, vs, &sh_s);
    const double s = sh_s;
    if (!(fabs(s) > 0.0) || !isfinite(cs[m])) {
      if (tid == 0 && blockIdx.x == 0 && flags) flags[0] |= 16;
    }
    if (blockIdx.x == 0) {
      const double is = 1.0 / s;
      for (int t = tid; t < k * k; t += 256) {
        const int i = t / k, j = t - i * k;
        double val;
        if (i < m && j < m)
          val = fma(us[i] * vs[j], is, Bs[i * 65 + j]);
        else if (i < m)
          val = -us[i] * is;
        else if (j < m)
          val = -vs[j] * is;
        else
          val = is;
        Bnext[i * 64 + j] = val;
      }
      if (tid < k) cnext[tid] = cs[tid];
    }
  }
  // The residual scan finds the winner of position k, which the next pass
  // (or the weights) takes.  A position that inherits its index needs none,
  // unless that index repeats one chosen before (then dg_choose falls back
  // to the scan): the same test as dg_choose's, on idx[0..k-2] and this
  // pass's winner of position k - 1 (idx[k - 1] is being written by block 0).
  if (forced) {
    const int f = forced[k];
    if (f >= 0 && f < N) {
      bool dup = false;
      for (int q = 0; q + 1 < k; ++q) dup |= (idx[q] == f);
      if (k > 0) dup |= (lwin == f);
      if (!dup) return;
    }
  }
  // residual coefficients: r_k = psi_k - sum_q c_q psi_q
  if (tid < 64) cf[tid] = (tid < k) ? -cs[tid] : ((tid == k) ? 1.0 : 0.0);
  __syncthreads();
  double best = -1.0;
  int bi = 0x7fffffff;
  auto take = [&](double v, int l) {
    if (v > best) {
      best = v;
      bi = l;
    }
  };
  // the two prefetched rows, then any further rows of the grid-stride loop
  if (l0 < N) {
    double r0 = 0.0, r1 = 0.0;
#pragma unroll
    for (int q = 0; q < DG_KR; q += 2) {
      r0 = fma(p0[q], cf[q], r0);
      r1 = fma(p0[q + 1], cf[q + 1], r1);
    }
    for (int q = DG_KR; q <= k; ++q) r0 = fma(Psi[(size_t)q * N + l0], cf[q], r0);
    take(fabs(r0 + r1), l0);
  }
  if (l1 < N) {
    double r0 = 0.0, r1 = 0.0;
#pragma unroll
    for (int q = 0; q < DG_KR; q += 2) {
      r0 = fma(p1[q], cf[q], r0);
      r1 = fma(p1[q + 1], cf[q + 1], r1);
    }
    for (int q = DG_KR; q <= k; ++q) r0 = fma(Psi[(size_t)q * N + l1], cf[q], r0);
    take(fabs(r0 + r1), l1);
  }
  for (int l = l1 + stride; l < N; l += stride) {
    double r0 = 0.0, r1 = 0.0;
    int q = 0;
    for (; q + 1 <= k; q += 2) {
      r0 = fma(Psi[(size_t)q * N + l], cf[q], r0);
      r1 = fma(Psi[(size_t)(q + 1) * N + l], cf[q + 1], r1);
    }
    if (q <= k) r0 = fma(Psi[(size_t)q * N + l], cf[q], r0);
    take(fabs(r0 + r1), l);
  }
  dg_wave_argmax(best, bi);
  if (lane == 0) {
    sv[w] = best;
    si[w] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    for (int q = 1; q < 4; ++q)
      if (sv[q] > best || (sv[q] == best && si[q] < bi)) {
        best = sv[q];
        bi = si[q];
      }
    bval[blockIdx.x] = best;
    bidx[blockIdx.x] = bi;
  }
}

// Last index l_{d-1} (winner of the last greedy pass) and the weights
// w = (P^T Psi)^{-T} Psi^T 1 of eq. grHDD (the factor m_p^{-1} M_q is applied
// in the gather).  With M_d^{-1} in the bordered form of the greedy passes
// (B = M_{d-1}^{-1}, u = c_{d-1}, v, s), and sigma = Psi^T 1 = (sigma', sigma_m):
//   g = (u.sigma' - sigma_m) / s,  w_i = (B^T sigma')_i + v_i g,  w_m = -g.
// colpart holds per-block column sums of Psi (ncp blocks).
__global__ void __launch_bounds__(256) deim_weights_kernel(
    const double* __restrict__ Psi, int N, int d, int* __restrict__ idx,
    const double* __restrict__ pval, const int* __restrict__ pidx, int nprev,
    const double* __restrict__ Bprev, const double* __restrict__ uprev,
    const double* __restrict__ colpart, int ncp, double* __restrict__ wout,
    int* __restrict__ flags, const int* __restrict__ forced) {
  __shared__ double Bs[64 * 65];
  __shared__ double us[64], ys[64], bs[64], cs[64], vs[64], sg[64];
  __shared__ double sh_s;
  __shared__ int lwin;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m = d - 1;
  for (int t = tid; t < m * m; t += 256) {
    const int i = t / m, j = t - i * m;
    Bs[i * 65 + j] = Bprev[i * 64 + j];
  }
  if (tid < 64) {
    us[tid] = (tid < m) ? uprev[tid] : 0.0;
    ys[tid] = 0.0;
    bs[tid] = 0.0;
    sg[tid] = 0.0;
  }
  if (w == 0) {
    int win = dg_choose(pval, pidx, nprev, forced, idx, d - 1, N);
    if (win < 0 || win >= N) {
      if (lane == 0 && flags) flags[0] |= 16;
      win = 0;
    }
    if (lane == 0) {
      lwin = win;
      idx[d - 1] = win;
    }
  }
  __syncthreads();
  // column sums of Psi: one wavefront per column, lane-strided partial sums
  // combined by a fixed butterfly
  for (int q = w; q < d; q += 4) {
    double s = 0.0;
    for (int b = lane; b < ncp; b += 64) s += colpart[(size_t)b * d + q];
    s = dg_wave_sum(s);
    if (lane == 0) sg[q] = s;
  }
  dg_border(Psi, N, d, -1, idx, lwin, Bs, us, ys, bs, cs, vs, &sh_s);
  if (tid < 64) {
    const double s = sh_s;
    double bt = 0.0;
    for (int i = 0; i < m; ++i) bt = fma(Bs[i * 65 + lane], sg[i], bt);   // (B^T sigma')_lane
    const double usg = dg_wave_sum((lane < m) ? us[lane] * sg[lane] : 0.0);
    const double g = (usg - sg[m]) / s;
    if (lane < m) wout[lane] = fma(vs[lane], g, bt);
    if (lane == m) wout[m] = -g;
    if (lane == 0 && (!(fabs(s) > 0.0) || !isfinite(g)) && flags) flags[0] |= 16;
  }
}

// (FP64 matrix-core tiles: the layout is described with mfma_f64_step.)
typedef mf4 mf_d4;
__device__ __forceinline__ mf_d4 mf_step(double a, double b, mf_d4 c) {
  return mfma_f64_step(a, b, c);
}

// DEIM basis Psi = Y M (N x d) from the snapshot slots (Y: N x P, column
// blocks of kin columns per slot) and M (P x d, ld ldM), computed as
// Psi^T = M^T Y^T on the matrix cores: per 16-row tile and 16 columns of
// Psi, 4-row slices of M^T (A, kept in registers) times 4 x 16 slices of Y^T
// (B: 16 consecutive rows of one column per 16 lanes).  Column sums of Psi
// per block into colpart[blockIdx][c] (fixed order: butterflies over the 16
// rows of a tile, tiles in order per lane, then the four wavefronts).
template <int NCB>
__global__ void __launch_bounds__(256) psi_mfma_kernel(RealList L, int kin, int N,
                                                       const double* __restrict__ M, int ldM,
                                                       int d, double* __restrict__ out,
                                                       double* __restrict__ colpart) {
  __shared__ double wsum[4][64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int P = L.count * kin;
  const int nks = (P + 3) / 4;
  const int li = lane & 15, lk = lane >> 4;
  // A operands: a[cb][ks] = M[4 ks + lk][16 cb + li] (zero outside)
  double a[NCB][16];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const int k = 4 * ks + lk, c = 16 * cb + li;
      a[cb][ks] = (k < P && c < d) ? M[(size_t)c * ldM + k] : 0.0;
    }
  // column pointers of Y for this lane's rows of B (k = 4 ks + lk)
  const double* yc[16];
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) {
    const int k = min(4 * ks + lk, P - 1);
    yc[ks] = L.ptr[k / kin] + (size_t)(k % kin) * N;
  }
  double cs[NCB][4];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) cs[cb][v] = 0.0;
  const int ntile = (N + 15) / 16;
  for (int t = blockIdx.x * 4 + w; t < ntile; t += gridDim.x * 4) {
    const int row = 16 * t + li;
    const int rowc = min(row, N - 1);
    double b[16];
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) b[ks] = yc[ks][rowc];
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) b[ks] = (row < N && 4 * ks + lk < P) ? b[ks] : 0.0;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      mf_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < 16; ++ks)
        if (ks < nks) acc = mf_step(a[cb][ks], b[ks], acc);
      // lane holds Psi[row 16 t + li][column 16 cb + 4 v + lk]
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * cb + 4 * v + lk;
        if (row < N && c < d) out[(size_t)c * N + row] = acc[v];
        cs[cb][v] += acc[v];   // zero for rows beyond N
      }
    }
  }
  // sums over the 16 rows of a tile (lanes with the same lk), then waves
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double x = cs[cb][v];
      x += bfly64<0>(x);
      x += bfly64<1>(x);
      x += bfly64<2>(x);
      x += bfly64<3>(x);
      if (li == 0) {
        const int c = 16 * cb + 4 * v + lk;
        if (c < 64) wsum[w][c] = x;
      }
    }
  __syncthreads();
  if (tid < d) {
    const double s = ((wsum[0][tid] + wsum[1][tid]) + wsum[2][tid]) + wsum[3][tid];
    colpart[(size_t)blockIdx.x * d + tid] = s;
  }
}

// Block of the snapshot Gram matrix, S = Ynew^T Yall (a <= 64 rows, b <= 64
// columns) over the rows [kb rk, (kb+1) rk), 16 rows of S at a time: per 16
// rows of Y, four 4-row slices of Ynew^T (A) and Yall (B, one 16-column
// block per accumulator); the four wavefronts' sums are added in order and
// written as this block's partial part[kb][ib * a + ia].
__global__ void __launch_bounds__(256) gram_mfma_kernel(RealList A, int ka, int a, RealList B,
                                                        int kbcols, int b, int N, int rk,
                                                        double* __restrict__ part,
                                                        const int* __restrict__ stop) {
  if (stop && *stop) return;
  __shared__ double red[4][16 * 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const double* pb[4];
  bool vb[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int jb = min(16 * cb + li, b - 1);
    pb[cb] = B.ptr[jb / kbcols] + (size_t)(jb % kbcols) * N;
    vb[cb] = 16 * cb + li < b;
  }
  const int ncb = (b + 15) / 16;
  const int r0 = blockIdx.x * rk, r1 = min(N, r0 + rk);
  const int nout = a * b;
  for (int i0 = 0; i0 < a; i0 += 16) {
    const int ia = min(i0 + li, a - 1);
    const double* pa = A.ptr[ia / ka] + (size_t)(ia % ka) * N;
    const bool va = i0 + li < a;
    mf_d4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = mf_d4{0.0, 0.0, 0.0, 0.0};
    for (int base = r0 + 16 * w; base < r1; base += 64) {
      // rows base + 4 s + lk, s = 0..3
      double av[4], bv[4][4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = base + 4 * s + lk;
        const int rowc = min(row, N - 1);
        const bool ok = row < r1;
        const double x = pa[rowc];
        av[s] = (ok && va) ? x : 0.0;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const double y = pb[cb][rowc];
          bv[cb][s] = (ok && vb[cb]) ? y : 0.0;
        }
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        if (cb < ncb)
#pragma unroll
          for (int s = 0; s < 4; ++s) acc[cb] = mf_step(av[s], bv[cb][s], acc[cb]);
    }
    // lane holds S[i0 + 4 v + lk][16 cb + li]
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w][(4 * v + lk) * 64 + 16 * cb + li] = acc[cb][v];
    __syncthreads();
    const int na = min(16, a - i0);
    for (int o = tid; o < na * b; o += 256) {
      const int i = o % na, j = o / na;
      const double sm = ((red[0][i * 64 + j] + red[1][i * 64 + j]) + red[2][i * 64 + j]) +
                        red[3][i * 64 + j];
      part[(size_t)blockIdx.x * nout + (size_t)j * a + i0 + i] = sm;
    }
    __syncthreads();
  }
}

// DEIM snapshot Lambda^0(X_r^i) Phi^i at every particle (Sec. 4.2.2, eq. Ydeim)
// for the parameters sub[0..psub): (1 - theta) Phi_j + theta Phi_{j+1}, written
// as column c of Y (N x psub).  The subset's coefficients (zero-padded to NC),
// factors and, when they fit (PH_LDS), potentials sit in LDS; positions use the
// deposit's operation order.
template <int NC, bool PH_LDS>
__global__ void __launch_bounds__(256) snapshot_kernel(const cplx* __restrict__ U, int N, int n,
                                                       const cplx* __restrict__ Z,
                                                       const int* __restrict__ sub, int psub,
                                                       int Nx, const double* __restrict__ factor,
                                                       const double* __restrict__ phi,
                                                       double* __restrict__ Y,
                                                       const int* __restrict__ stop) {
  if (stop && *stop) return;
  extern __shared__ double smem[];
  cplx* Zs = reinterpret_cast<cplx*>(smem);                 // [psub][NC]
  double* fs = reinterpret_cast<double*>(Zs + psub * NC);    // [psub]
  double* ph = fs + psub;                                    // [psub][Nx] (PH_LDS)
  const int tid = threadIdx.x;
  for (int t = tid; t < psub * NC; t += 256) {
    const int c = t / NC, k = t % NC;
    Zs[t] = (k < n) ? Z[(size_t)sub[c] * n + k] : mk(0.0, 0.0);
  }
  for (int c = tid; c < psub; c += 256) fs[c] = factor[sub[c]];
  if (PH_LDS)
    for (int t = tid; t < psub * Nx; t += 256) {
      const int c = t / Nx, j = t % Nx;
      ph[t] = phi[(size_t)sub[c] * Nx + j];
    }
  __syncthreads();
  const int l = blockIdx.x * 256 + tid;
  if (l >= N) return;
  cplx u[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) u[k] = (k < n) ? U[(size_t)k * N + l] : mk(0.0, 0.0);
  for (int c = 0; c < psub; ++c) {
    const cplx* zc = Zs + c * NC;
    double x0 = 0.0, x1 = 0.0;
#pragma unroll
    for (int k = 0; k < NC; k += 2) {
      x0 = fma(u[k].re, zc[k].re, x0);
      x0 = fma(-u[k].im, zc[k].im, x0);
      if (k + 1 < NC) {
        x1 = fma(u[k + 1].re, zc[k + 1].re, x1);
        x1 = fma(-u[k + 1].im, zc[k + 1].im, x1);
      }
    }
    int j;
    double th;
    cell_of(x0 + x1, fs[c], Nx, j, th);
    const int j1 = (j + 1 == Nx) ? 0 : j + 1;
    const double* pc = PH_LDS ? ph + c * Nx : phi + (size_t)sub[c] * Nx;
    Y[(size_t)c * N + l] = (1.0 - th) * pc[j] + th * pc[j1];
  }
}


// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
bool fused_gradient_ok(int n) { return n <= 16; }

static int fused_nc(int n) { return nc_even(n); }

namespace {
// shapes set by set_gather_project_shape, by (N, p, Nx, column count)
std::mutex gp_shape_mu;
std::map<std::array<int, 4>, GpShape> gp_shapes;

// LDS the kernel may take beyond its static arrays (the attribute call of
// ALLOW_BIG_LDS raises the cap to the CU's 160 KB)
constexpr size_t kGpLdsMax = 150 * 1024;

size_t gp_lds_bytes(const GpShape& sh, int Nx, int nc) {
  const int pt = 16 * sh.cbn;
  const int wv = (sh.cbn <= 2) ? 8 : 4;
  const int mt = (2 * nc + 15) / 16;
  const size_t et = sh.et_lds ? (size_t)pt * Nx * sizeof(double) : 0;
  const size_t red = (size_t)wv * 16 * mt * pt * sizeof(double) + (size_t)wv * pt * sizeof(double);
  return std::max(et, red);
}
}  // namespace

// the built-in rule: parameter tiles of 16 CBN with their field rows in LDS
// (CBN as large as a 72 KB budget allows, at most 4; without room for even
// 16 rows, tiles of 64 with the table read from global memory), and two
// blocks per CU (512 row blocks on 256 CUs)
GpShape gather_project_shape(int N, int p, int Nx, int n, size_t part_cap) {
  const int nc = fused_nc(n);
  {
    std::lock_guard<std::mutex> lk(gp_shape_mu);
    auto it = gp_shapes.find({N, p, Nx, nc});
    if (it != gp_shapes.end()) return it->second;
  }
  (void)part_cap;
  const size_t budget = 72 * 1024;
  GpShape sh{4, true, 512};
  while (sh.cbn > 1 && (size_t)16 * sh.cbn * Nx * sizeof(double) > budget) sh.cbn /= 2;
  sh.et_lds = (size_t)16 * sh.cbn * Nx * sizeof(double) <= budget;
  if (!sh.et_lds) sh.cbn = 4;
  return sh;
}

std::vector<GpShape> gather_project_shapes(int N, int p, int Nx, int n, size_t part_cap) {
  const int nc = fused_nc(n);
  const int rec = n * p + p;
  const int cap = (int)(part_cap / (size_t)rec);
  std::vector<GpShape> out;
  std::vector<std::array<int, 3>> seen;  // (cbn, et, effective row blocks)
  for (int cbn : {1, 2, 4})
    for (bool et : {true, false})
      for (int nbm : {256, 512, 1024}) {
        const GpShape sh{cbn, et, nbm};
        if (gp_lds_bytes(sh, Nx, nc) > kGpLdsMax) continue;
        if (cbn > 1 && 16 * (cbn / 2) >= p) continue;  // a narrower tile already holds p
        const int eff = std::max(1, std::min(std::min(nbm, (N + 63) / 64), cap));
        const std::array<int, 3> k{cbn, et ? 1 : 0, eff};
        if (std::find(seen.begin(), seen.end(), k) != seen.end()) continue;
        seen.push_back(k);
        out.push_back(sh);
      }
  return out;
}

void set_gather_project_shape(int N, int p, int Nx, int n, const GpShape* shape) {
  std::lock_guard<std::mutex> lk(gp_shape_mu);
  const std::array<int, 4> key{N, p, Nx, fused_nc(n)};
  if (shape)
    gp_shapes[key] = *shape;
  else
    gp_shapes.erase(key);
}

void launch_gather_project(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p,
                           int Nx, const double* factor, const double* e, double qm,
                           const int* active, bool want_colsq, cplx* part, size_t part_cap,
                           cplx* g, double* colsq, const cplx* G12, const int* gate) {
  const int nc = fused_nc(n);
  const int rec = n * p + p;
  const GpShape shape = gather_project_shape(N, p, Nx, n, part_cap);
  // at least 64 rows per block, at most nb_max blocks (all resident at once:
  // every CU gets the same share), partials within part_cap
  int nb = (N + 63) / 64;
  if (nb > shape.nb_max) nb = shape.nb_max;
  const int cap = (int)(part_cap / (size_t)rec);
  if (nb > cap) nb = cap;
  if (nb < 1) nb = 1;
  const int rpb = (N + nb - 1) / nb;
  nb = (N + rpb - 1) / rpb;
  const int cbn = shape.cbn;
  const bool et_lds = shape.et_lds;
  const int pt = 16 * cbn;
  const int ntile = (p + pt - 1) / pt;
  const size_t et_bytes = et_lds ? (size_t)pt * Nx * sizeof(double) : 0;
  // eight wavefronts per block on one field table when the tile is narrow
  // (more wavefronts per SIMD for the same LDS), else four; the wavefront
  // sums reuse the table's space: WV x 16 MT x PT + WV x PT doubles
  const int wv = (cbn <= 2) ? 8 : 4;
  const int mt = (2 * nc + 15) / 16;
  const size_t red_bytes =
      (size_t)wv * 16 * mt * pt * sizeof(double) + (size_t)wv * pt * sizeof(double);
  const size_t sh = std::max(et_bytes, red_bytes);
  dim3 grid(ntile, nb);
#define GPM(NCV, CBV, ETV)                                                                  \
  {                                                                                        \
    constexpr int WVV = (CBV <= 2) ? 8 : 4;                                                \
    ALLOW_BIG_LDS((gather_project_mfma_kernel<NCV, CBV, ETV, WVV>));                       \
    hipLaunchKernelGGL((gather_project_mfma_kernel<NCV, CBV, ETV, WVV>), grid, dim3(64 * WVV), \
                       sh, s, U, N, n, Z, p, Nx, rpb, factor, e, qm, active, rec,           \
                       want_colsq ? 1 : 0, part, gate);                                     \
  }
#define GPM_NC(CBV, ETV)                \
  switch (nc) {                         \
    case 4: GPM(4, CBV, ETV); break;    \
    case 5: GPM(5, CBV, ETV); break;    \
    case 6: GPM(6, CBV, ETV); break;    \
    case 7: GPM(7, CBV, ETV); break;    \
    case 8: GPM(8, CBV, ETV); break;    \
    case 12: GPM(12, CBV, ETV); break;  \
    default: GPM(16, CBV, ETV); break;  \
  }
  if (et_lds) {
    if (cbn == 4) {
      GPM_NC(4, true)
    } else if (cbn == 2) {
      GPM_NC(2, true)
    } else {
      GPM_NC(1, true)
    }
  } else {
    if (cbn == 4) {
      GPM_NC(4, false)
    } else if (cbn == 2) {
      GPM_NC(2, false)
    } else {
      GPM_NC(1, false)
    }
  }
#undef GPM_NC
#undef GPM
  const int nout = want_colsq ? rec : n * p;
  hipLaunchKernelGGL(reduce_partials2_kernel, dim3((nout + 3) / 4), dim3(256), 0, s, part, nb, rec,
                     n * p, nout, g, colsq, gate, G12, Z, n);
}


void launch_gather_xi(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                      const double* factor, const double* e, double qm, const cplx* Q,
                      const cplx* MU, double h, cplx* out, const cplx* g) {
  const int nc = fused_nc(n);
  // 256 rows per block (four wavefronts of 64)
  dim3 grid((N + 255) / 256);
#define GXM(NCV)                                                                               \
  hipLaunchKernelGGL(gather_xi_mfma_kernel<NCV>, grid, dim3(256), 0, s, U, N, n, Z, p, Nx, factor, \
                     e, qm, Q, MU, g, h, out)
  switch (nc) {
    case 4: GXM(4); break;
    case 5: GXM(5); break;
    case 6: GXM(6); break;
    case 7: GXM(7); break;
    case 8: GXM(8); break;
    case 12: GXM(12); break;
    default: GXM(16); break;
  }
#undef GXM
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
                        double* X, double* V, const int* rows, int nrows) {
  const int nout = rows ? nrows : N;
  if (nout <= 0) return;
  int nc = nc_bucket(n);
  dim3 grid((nout + 255) / 256);
#define RC(NCV) \
  hipLaunchKernelGGL(reconstruct_kernel<NCV>, grid, dim3(256), 0, s, U, N, n, Z, p, X, V, rows, nout)
  switch (nc) {
    case 4: RC(4); break;
    case 8: RC(8); break;
    case 16: RC(16); break;
    default: RC(32); break;
  }
#undef RC
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

bool launch_rowgemm_gram(hipStream_t s, const RowTerms& T, int N, int m, cplx* out, cplx* part,
                         size_t part_cap, cplx* Gram, const cplx* pre, int kp) {
  const int nb = (N + 255) / 256;
  if (!pre) kp = 0;
  const int g = kp + m;
  if (m > 8 || kp > 8 || (size_t)nb * g * g > part_cap) return false;
  size_t sh = 0;
  for (int q = 0; q < T.count; ++q) sh += (size_t)T.k[q] * m * sizeof(cplx);
  const dim3 grid(nb), blk(256);
  ALLOW_BIG_LDS((rowgemm_gram_kernel<4, true>));
  ALLOW_BIG_LDS((rowgemm_gram_kernel<8, true>));
  ALLOW_BIG_LDS((rowgemm_gram_kernel<4, false>));
  ALLOW_BIG_LDS((rowgemm_gram_kernel<8, false>));
  if (pre) {
    if (m <= 4 && kp <= 4)
      hipLaunchKernelGGL((rowgemm_gram_kernel<4, true>), grid, blk, sh, s, T, N, m, out, pre, kp,
                         part);
    else
      hipLaunchKernelGGL((rowgemm_gram_kernel<8, true>), grid, blk, sh, s, T, N, m, out, pre, kp,
                         part);
  } else {
    if (m <= 4)
      hipLaunchKernelGGL((rowgemm_gram_kernel<4, false>), grid, blk, sh, s, T, N, m, out, pre, 0,
                         part);
    else
      hipLaunchKernelGGL((rowgemm_gram_kernel<8, false>), grid, blk, sh, s, T, N, m, out, pre, 0,
                         part);
  }
  const int nout = g * g;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((nout + 3) / 4), dim3(256), 0, s, part, nb, nout,
                     Gram);
  return true;
}

static void rowgemm_launch(hipStream_t s, const RowTerms& T, int N, int m, cplx* out, int accum) {
  size_t sh = 0;
  for (int q = 0; q < T.count; ++q) sh += (size_t)T.k[q] * m * sizeof(cplx);
  dim3 grid((N + 255) / 256);
  int mc = nc_bucket(m);
  ALLOW_BIG_LDS(rowgemm_kernel<4>);
  ALLOW_BIG_LDS(rowgemm_kernel<8>);
  ALLOW_BIG_LDS(rowgemm_kernel<16>);
  ALLOW_BIG_LDS(rowgemm_kernel<32>);
  switch (mc) {
    case 4: hipLaunchKernelGGL(rowgemm_kernel<4>, grid, dim3(256), sh, s, T, N, m, out, accum); break;
    case 8: hipLaunchKernelGGL(rowgemm_kernel<8>, grid, dim3(256), sh, s, T, N, m, out, accum); break;
    case 16: hipLaunchKernelGGL(rowgemm_kernel<16>, grid, dim3(256), sh, s, T, N, m, out, accum); break;
    default: hipLaunchKernelGGL(rowgemm_kernel<32>, grid, dim3(256), sh, s, T, N, m, out, accum); break;
  }
}

// The M matrices of all terms are staged in LDS.  When they do not fit
// (a wide first input, as G~ Q over many parameters), the terms are taken
// one at a time and a wide term in slices of its columns, each launch
// adding to the output (a slice of M_q is a row range, read in place with
// its leading dimension).
void launch_rowgemm(hipStream_t s, const RowTerms& T, int N, int m, cplx* out) {
  const size_t lds_cap = 144 * 1024;
  size_t sh = 0;
  for (int q = 0; q < T.count; ++q) sh += (size_t)T.k[q] * m * sizeof(cplx);
  if (sh <= lds_cap) {
    rowgemm_launch(s, T, N, m, out, 0);
    return;
  }
  const int kmax = (int)(lds_cap / ((size_t)m * sizeof(cplx)));
  int accum = 0;
  for (int q = 0; q < T.count; ++q) {
    for (int k0 = 0; k0 < T.k[q]; k0 += kmax) {
      const int kc = std::min(kmax, T.k[q] - k0);
      RowTerms U{};
      U.count = 1;
      U.in[0] = T.in[q] + (size_t)k0 * N;
      U.k[0] = kc;
      U.M[0] = T.M[q];
      // rows k0 .. k0 + kc of M_q, read in place with its leading dimension
      U.M[0] = T.M[q] + k0;
      U.ld[0] = T.ld[q] ? T.ld[q] : T.k[q];
      rowgemm_launch(s, U, N, m, out, accum);
      accum = 1;
    }
  }
}

void launch_deim_gather(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                        const double* factor, const double* e, double qm, const int* idx,
                        const double* w, int d, const int* active, cplx* gF, const int* gate,
                        const DeimStartArgs* start) {
  DeimStartArgs st{};
  if (start) st = *start;
  hipLaunchKernelGGL(deim_gather_kernel, dim3(p), dim3(64), 0, s, U, N, n, Z, p, Nx, factor, e,
                     qm, idx, w, d, active, gF, gate, st);
}



// Sum the partials of a real product and scatter the a x b result into the
// symmetric P x P matrix S at rows r0.. (and the transpose at columns r0..).
__global__ void __launch_bounds__(256) reduce_gram_block_kernel(const double* __restrict__ part,
                                                                int nkb, int a, int b, int P,
                                                                int r0, double* __restrict__ S,
                                                                const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int lane = threadIdx.x & 63;
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nout = a * b;
  if (o >= nout) return;
  double s = 0.0;
  // eight partials of a lane in flight at once (clamped loads, masked adds)
  for (int k0 = lane; k0 < nkb; k0 += 8 * 64) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)min(k0 + 64 * u, nkb - 1) * nout + o];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += (k0 + 64 * u < nkb) ? v[u] : 0.0;
  }
  for (int w = 32; w > 0; w >>= 1) s += __shfl_xor(s, w, 64);
  if (lane == 0) {
    const int ia = o % a, ib = o / a;
    S[(size_t)ib * P + r0 + ia] = s;   // row r0+ia, column ib
    S[(size_t)(r0 + ia) * P + ib] = s; // transpose
  }
}

void launch_gram_block_real(hipStream_t s, const double* Ynew, const double* const* slots,
                            int nslots, int psub, int N, int r0, int nkb_cap, double* part,
                            double* S, const int* stop) {
  RealList A{}, B{};
  A.ptr[0] = Ynew;
  A.count = 1;
  for (int q = 0; q < nslots; ++q) B.ptr[q] = slots[q];
  B.count = nslots;
  const int a = psub, b = psub * nslots;
  int nkb = (N + 127) / 128;
  if (nkb > 512) nkb = 512;
  const int cap = nkb_cap / (a * b);
  if (nkb > cap) nkb = cap;
  if (nkb < 1) nkb = 1;
  const int rk = (N + nkb - 1) / nkb;
  nkb = (N + rk - 1) / rk;
  hipLaunchKernelGGL(gram_mfma_kernel, dim3(nkb), dim3(256), 0, s, A, psub, a, B, psub, b, N, rk,
                     part, stop);
  hipLaunchKernelGGL(reduce_gram_block_kernel, dim3((a * b + 3) / 4), dim3(256), 0, s, part, nkb, a,
                     b, b, r0, S, stop);
}

void launch_snapshot(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, const int* sub,
                     int psub, int Nx, const double* factor, const double* phi, double* Y,
                     const int* stop) {
  const int nc = (n <= 16) ? fused_nc(n) : 32;
  const size_t base = (size_t)psub * nc * sizeof(cplx) + (size_t)psub * sizeof(double);
  const size_t phb = (size_t)psub * Nx * sizeof(double);
  const bool ph_lds = base + phb <= 96 * 1024;
  const size_t sh = base + (ph_lds ? phb : 0);
  dim3 grid((N + 255) / 256);
#define SN(NCV, PV)                                                                          \
  ALLOW_BIG_LDS((snapshot_kernel<NCV, PV>));                                               \
  hipLaunchKernelGGL((snapshot_kernel<NCV, PV>), grid, dim3(256), sh, s, U, N, n, Z, sub, psub, \
                     Nx, factor, phi, Y, stop)
  if (ph_lds) {
    switch (nc) {
      case 4: SN(4, true); break;
      case 5: SN(5, true); break;
      case 6: SN(6, true); break;
      case 7: SN(7, true); break;
      case 8: SN(8, true); break;
      case 12: SN(12, true); break;
      case 16: SN(16, true); break;
      default: SN(32, true); break;
    }
  } else {
    switch (nc) {
      case 4: SN(4, false); break;
      case 5: SN(5, false); break;
      case 6: SN(6, false); break;
      case 7: SN(7, false); break;
      case 8: SN(8, false); break;
      case 12: SN(12, false); break;
      case 16: SN(16, false); break;
      default: SN(32, false); break;
    }
  }
#undef SN
}

int psi_blocks(int N) {
  int nb = (N + 255) / 256;
  return nb > 512 ? 512 : nb;
}

void launch_psi_colsum(hipStream_t s, const double* const* in, int nin, int kin, int N,
                       const double* M, int ldM, int d, double* out, double* colpart) {
  RealList L{};
  for (int q = 0; q < nin; ++q) L.ptr[q] = in[q];
  L.count = nin;
  dim3 grid(psi_blocks(N));
  if (d <= 16)
    hipLaunchKernelGGL(psi_mfma_kernel<1>, grid, dim3(256), 0, s, L, kin, N, M, ldM, d, out, colpart);
  else if (d <= 32)
    hipLaunchKernelGGL(psi_mfma_kernel<2>, grid, dim3(256), 0, s, L, kin, N, M, ldM, d, out, colpart);
  else
    hipLaunchKernelGGL(psi_mfma_kernel<4>, grid, dim3(256), 0, s, L, kin, N, M, ldM, d, out, colpart);
}

void launch_deim_greedy(hipStream_t s, const double* Psi, int N, int k, int* idx,
                        const double* pval, const int* pidx, int nprev, int nblk, double* bval,
                        int* bidx, const double* Bprev, const double* uprev, double* Bnext,
                        double* cnext, int* flags, const int* forced) {
  hipLaunchKernelGGL(deim_greedy_kernel, dim3(nblk), dim3(256), 0, s, Psi, N, k, idx, pval, pidx,
                     nprev, bval, bidx, Bprev, uprev, Bnext, cnext, flags, forced);
}

void launch_deim_weights(hipStream_t s, const double* Psi, int N, int d, int* idx,
                         const double* pval, const int* pidx, int nprev, const double* Bprev,
                         const double* uprev, const double* colpart, int ncp, double* w,
                         int* flags, const int* forced) {
  hipLaunchKernelGGL(deim_weights_kernel, dim3(1), dim3(256), 0, s, Psi, N, d, idx, pval, pidx,
                     nprev, Bprev, uprev, colpart, ncp, w, flags, forced);
}

// Rotation of the DEIM basis between two operators: per block, the partial
// dot products psi_k^new . psi_k^old over its rows (d columns), summed in a
// fixed order by deim_forced_kernel.
__global__ void __launch_bounds__(256) psi_rot_kernel(const double* __restrict__ Pn,
                                                      const double* __restrict__ Po, int N, int d,
                                                      double* __restrict__ part) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  __shared__ double ws4[4][64];
  for (int k = 0; k < d; ++k) {
    double a = 0.0;
    for (int l = blockIdx.x * 256 + tid; l < N; l += gridDim.x * 256)
      a = fma(Pn[(size_t)k * N + l], Po[(size_t)k * N + l], a);
    a = dg_wave_sum(a);
    if (lane == 0) ws4[w][k & 63] = a;
    __syncthreads();
    if (tid == 0) part[(size_t)blockIdx.x * d + k] = ((ws4[0][k & 63] + ws4[1][k & 63]) +
                                                      ws4[2][k & 63]) + ws4[3][k & 63];
    __syncthreads();
  }
}

// The adaptive update's inherited indices: |psi_k^new . psi_k^old| (block
// partials summed in order); the n_up smallest (ties to the smaller
// position) are chosen again (forced = -1), the other positions inherit
// their previous index (forced = idx_old[k]).
__global__ void deim_forced_kernel(const double* __restrict__ part, int nb, int d, int n_up,
                                   const int* __restrict__ idx_old, int* __restrict__ forced,
                                   const int* __restrict__ stop) {
  if (stop && *stop) return;
  __shared__ double rot[64];
  const int k = threadIdx.x;
  if (k < d) {
    double a = 0.0;
    for (int b = 0; b < nb; ++b) a += part[(size_t)b * d + k];
    rot[k] = fabs(a);
  }
  __syncthreads();
  if (k < d) {
    // rank of position k in increasing rotation measure (stable)
    int rank = 0;
    for (int q = 0; q < d; ++q) rank += (rot[q] < rot[k]) || (rot[q] == rot[k] && q < k);
    forced[k] = (rank < n_up) ? -1 : idx_old[k];
  }
}

void launch_deim_forced(hipStream_t s, const double* Pn, const double* Po, int N, int d, int n_up,
                        const int* idx_old, double* part, int* forced, const int* stop) {
  const int nb = psi_blocks(N);
  hipLaunchKernelGGL(psi_rot_kernel, dim3(nb), dim3(256), 0, s, Pn, Po, N, d, part);
  hipLaunchKernelGGL(deim_forced_kernel, dim3(1), dim3(64), 0, s, part, nb, d, n_up, idx_old,
                     forced, stop);
}
