// Particle-to-grid kernels of the periodic P1 particle-in-cell model
// (paper Sec. 2.1): charge deposit, Poisson solve, field, and the fused
// Stormer-Verlet push of the full-order model (eq. sv_full_order).
#include "common.h"
#include "kernels.h"

// ---------------------------------------------------------------------------
// Deposit from explicit positions X (N x p, column-major).
//
// Grid (nrb, ntiles): block (rb, tile) owns rows [rb*rpb, (rb+1)*rpb) and the
// parameters [tile*pt, tile*pt + pt).  The block accumulates the unit weights
// (1 - theta) and theta into an LDS histogram of pt x Nx doubles with FP64 LDS
// atomics and writes it to part[rb][i][j]; the Poisson kernel sums the row
// blocks in a fixed order and scales by q w_i.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(512) deposit_x_kernel(const double* __restrict__ X, int N, int p,
                                                        int Nx, int pt, int rpb,
                                                        const double* __restrict__ factor,
                                                        double* __restrict__ part) {
  extern __shared__ double hist[];
  const int rb = blockIdx.x;
  const int p0 = blockIdx.y * pt;
  const int np = min(pt, p - p0);
  for (int t = threadIdx.x; t < np * Nx; t += blockDim.x) hist[t] = 0.0;
  __syncthreads();
  const int r0 = rb * rpb;
  const int r1 = min(N, r0 + rpb);
  for (int i = 0; i < np; ++i) {
    const double f = factor[p0 + i];
    const double* Xi = X + (size_t)(p0 + i) * N;
    double* hi = hist + i * Nx;
    for (int l = r0 + threadIdx.x; l < r1; l += blockDim.x) {
      int j;
      double th;
      cell_of(Xi[l], f, Nx, j, th);
      int j1 = (j + 1 == Nx) ? 0 : j + 1;
      lds_add(hi + j, 1.0 - th);
      lds_add(hi + j1, th);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < np * Nx; t += blockDim.x)
    part[((size_t)rb * p + p0) * Nx + t] = hist[t];
}

// ---------------------------------------------------------------------------
// Reduced-model deposit: positions are reconstructed on the fly,
// x_{l,i} = Re( sum_k U~[l,k] Z~[k,i] ), and never written to memory.
// A thread holds the n complex basis entries of DEP_ROWS particle rows in
// registers (loaded together, at clamped indices and masked, so that no
// load sits behind a branch); the parameter loop runs outside the rows, so
// one set of coefficient loads (uniform: scalar loads) serves every row of
// the thread and the LDS queue holds nothing but the histogram atomics.
// Parameters whose `active` flag is 0 are skipped (frozen fixed-point
// columns).  Small column counts run 16 wavefronts per block: one block per
// CU is the usual launch, and the LDS atomics need that many in flight.
// Per cell c the block counts its particles (32-bit integer atomics) and
// sums their theta (FP64 atomics); the weight of node j is then
// count_j - T_j + T_{j-1} (the (1 - theta) of the particles in cell j and
// the theta of those in cell j - 1): one 64-bit atomic per particle instead
// of two, and a 32-bit one, which the LDS serves with fewer bank conflicts.
// ---------------------------------------------------------------------------
template <int NC>
constexpr int deposit_rom_threads() {
  return (NC <= 8) ? 1024 : 512;
}
template <int NC>
constexpr int deposit_rom_rows() {
  return (NC <= 16) ? 2 : 1;
}

template <int NC>
__global__ void __launch_bounds__(deposit_rom_threads<NC>()) deposit_rom_kernel(
    const cplx* __restrict__ U, int N, int n, const cplx* __restrict__ Z, int p, int Nx, int pt,
    int rpb, const double* __restrict__ factor, const int* __restrict__ active,
    double* __restrict__ part, const int* __restrict__ gate, int* __restrict__ fold, int det) {
  if (gate && gate[0] == 0) return;
  if (fold && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    // end-of-step bookkeeping of the status words (the step's kernels are
    // done): the error word of the DEIM chain of the step (3) is folded into
    // the step's chain word (2) and cleared; the stop word (12) of the chain
    // enqueued next is set when this step failed
    const int tail = fold[2] | fold[3];
    fold[2] = tail;
    fold[3] = 0;
    fold[12] = fold[0] | tail;
  }
  constexpr int R = deposit_rom_rows<NC>();
  extern __shared__ double hist[];                                    // theta sums, pt * Nx
  unsigned* cnt = reinterpret_cast<unsigned*>(hist + (size_t)pt * Nx);  // counts, pt * Nx
  const int rb = blockIdx.x;
  const int p0 = blockIdx.y * pt;
  const int np = min(pt, p - p0);
  for (int t = threadIdx.x; t < np * Nx; t += blockDim.x) {
    hist[t] = 0.0;
    cnt[t] = 0u;
  }
  __syncthreads();
  const int r0 = rb * rpb;
  const int r1 = min(N, r0 + rpb);
  const int bs = blockDim.x;
  for (int lb = r0; lb < r1; lb += R * bs) {
    cplx u[R][NC];
    bool ok[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int l = lb + r * bs + (int)threadIdx.x;
      ok[r] = l < r1;
      const int lc = min(l, r1 - 1);
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const cplx v = U[(size_t)min(k, n - 1) * N + lc];
        const double m = (k < n) ? 1.0 : 0.0;  // columns k >= n are zero
        u[r][k] = mk(v.re * m, v.im * m);
      }
    }
    for (int i = 0; i < np; ++i) {
      if (active && !active[p0 + i]) continue;
      cplx z[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const cplx a = Z[(size_t)(p0 + i) * n + min(k, n - 1)];
        z[k] = (k < n) ? a : mk(0.0, 0.0);
      }
      const double f = factor[p0 + i];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // two partial sums (even and odd columns), as in every kernel that
        // locates particles, so that the cells agree bit for bit
        double x0 = 0.0, x1 = 0.0;
#pragma unroll
        for (int k = 0; k < NC; k += 2) {
          x0 = fma(u[r][k].re, z[k].re, x0);
          x0 = fma(-u[r][k].im, z[k].im, x0);
          if (k + 1 < NC) {
            x1 = fma(u[r][k + 1].re, z[k + 1].re, x1);
            x1 = fma(-u[r][k + 1].im, z[k + 1].im, x1);
          }
        }
        int j;
        double th;
        cell_of(x0 + x1, f, Nx, j, th);
        if (ok[r]) {
          __hip_atomic_fetch_add(cnt + i * Nx + j, 1u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
          if (det)
            __hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(hist) + i * Nx + j,
                                   __double2ull_rn(th * 0x1p40), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
          else
            lds_add(hist + i * Nx + j, th);
        }
      }
    }
  }
  __syncthreads();
  if (det) {
    // each integer sum becomes a double in place (one rounding each)
    const unsigned long long* ih = reinterpret_cast<const unsigned long long*>(hist);
    for (int t = threadIdx.x; t < np * Nx; t += blockDim.x) {
      const double v = __ull2double_rn(ih[t]) * 0x1p-40;
      hist[t] = v;
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < np * Nx; t += blockDim.x) {
    const int i = t / Nx, j = t - i * Nx;
    if (active && !active[p0 + i]) continue;
    const int jm = (j == 0) ? Nx - 1 : j - 1;
    part[((size_t)rb * p + p0) * Nx + t] = ((double)cnt[t] - hist[t]) + hist[i * Nx + jm];
  }
}

// ---------------------------------------------------------------------------
// The same deposit with the positions formed on the FP64 matrix cores
// (PosRows / pos_tile, as the gather-projection forms them, so that both see
// the same cells): a tile of PT <= 16 parameters per block (one B operand;
// lanes past PT idle), each of the 16 wavefronts taking 16-row tiles in
// turn; lane li + 16 lk ends with the positions of rows 4 v + lk for
// parameter li and adds them to the block's count and theta tables.  The
// operands of the next row tile are loaded while the current one is
// deposited.
// ---------------------------------------------------------------------------
int deposit_tile_params(int Nx) {
  // count and theta tables of PT parameters within 128 KB of LDS
  int pt = (int)((size_t)128 * 1024 / ((size_t)Nx * (sizeof(double) + sizeof(unsigned))));
  return pt < 1 ? 1 : (pt > 16 ? 16 : pt);
}

template <int NC>
__global__ void __launch_bounds__(1024) deposit_rom_mfma_kernel(
    const cplx* __restrict__ U, int N, int n, const cplx* __restrict__ Z, int p, int Nx, int PT,
    int rpb, const double* __restrict__ factor, const int* __restrict__ active,
    double* __restrict__ part, const int* __restrict__ gate, int* __restrict__ fold, int det) {
  if (gate && gate[0] == 0) return;
  if (fold && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    // end-of-step bookkeeping of the status words, as in deposit_rom_kernel
    const int tail = fold[2] | fold[3];
    fold[2] = tail;
    fold[3] = 0;
    fold[12] = fold[0] | tail;
  }
  constexpr int KS = (2 * NC + 3) / 4;
  extern __shared__ double hist[];                                    // theta sums, PT * Nx
  unsigned* cnt = reinterpret_cast<unsigned*>(hist + (size_t)PT * Nx);  // counts, PT * Nx
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int rb = blockIdx.x;
  const int p0 = blockIdx.y * PT;
  const int np = min(PT, p - p0);
  for (int t = tid; t < np * Nx; t += blockDim.x) {
    hist[t] = 0.0;
    cnt[t] = 0u;
  }
  const int c = p0 + min(li, np - 1);
  const bool on = li < np && (!active || active[c]);  // (np <= PT <= 16)
  const double fac = factor[c];
  double bz[KS];
  pos_coefs<KS>(Z, n, NC, c, on, lk, bz);
  PosRows<KS> pr;
  pr.setup(U, N, n, NC, lk);
  __syncthreads();
  const int r0 = rb * rpb;
  const int r1 = min(N, r0 + rpb);
  double a[KS], an[KS];
  pr.load(min(r0 + 16 * w + li, r1 - 1), a);
  for (int t0 = r0 + 16 * w; t0 < r1; t0 += 16 * nw) {
    pr.load(min(t0 + 16 * nw + li, r1 - 1), an);
    const mf4 X = pos_tile<KS>(a, bz);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int j;
      double th;
      cell_of(X[v], fac, Nx, j, th);
      if (on && t0 + 4 * v + lk < r1) {
        __hip_atomic_fetch_add(cnt + li * Nx + j, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        if (det)
          __hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(hist) + li * Nx + j,
                                 __double2ull_rn(th * 0x1p40), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        else
          lds_add(hist + li * Nx + j, th);
      }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a[ks] = an[ks];
  }
  __syncthreads();
  if (det) {
    // each integer sum becomes a double in place (one rounding each)
    const unsigned long long* ih = reinterpret_cast<const unsigned long long*>(hist);
    for (int t = tid; t < np * Nx; t += blockDim.x) {
      const double v = __ull2double_rn(ih[t]) * 0x1p-40;
      hist[t] = v;
    }
    __syncthreads();
  }
  for (int t = tid; t < np * Nx; t += blockDim.x) {
    const int i = t / Nx, j = t - i * Nx;
    if (active && !active[p0 + i]) continue;
    const int jm = (j == 0) ? Nx - 1 : j - 1;
    part[((size_t)rb * p + p0) * Nx + t] = ((double)cnt[t] - hist[t]) + hist[i * Nx + jm];
  }
}

// ---------------------------------------------------------------------------
// Poisson solve (eq. PoissonSystem) for one parameter per block.
//
// rho_j = q w_i * (sum of the row-block partials) + h_i (P1 load vector of
// the unit background).  The periodic P1 stiffness (1/h) circ(-1, 2, -1) is a
// second difference: with e_j = (Phi_{j+1} - Phi_j)/h, (L Phi)_j = e_{j-1} - e_j,
// so e is minus the prefix sum S of the zero-mean charge plus the constant
// that makes sum_j e_j = 0 (periodic Phi): e_j = mean(S) - S_j.  Phi follows
// from Phi_{j+1} = Phi_j + h e_j and the zero-mean gauge.  This is the exact
// pseudo-inverse solution, in O(Nx).  Energy E_i = Phi^T rho / (2 m w_i).
// ---------------------------------------------------------------------------
// exclusive prefix sum over the 64 lanes of a wavefront: Hillis-Steele
// inside rows of 16 by row shifts, the row totals carried by the row
// broadcasts of lanes 15 and 31, then the inclusive sums moved up one lane
__device__ __forceinline__ double wave_exclusive_scan(double v) {
  v += dpp64<0x111, 0xf>(v);  // row_shr:1
  v += dpp64<0x112, 0xf>(v);  // row_shr:2
  v += dpp64<0x114, 0xf>(v);  // row_shr:4
  v += dpp64<0x118, 0xf>(v);  // row_shr:8
  v += dpp64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const double up = __shfl_up(v, 1, 64);
  return ((threadIdx.x & 63) == 0) ? 0.0 : up;
}

constexpr int POISSON_THREADS = 512;
constexpr int POISSON_PER_LANE = SYMROM_MAX_NX / 64;  // nodes per lane in the solve

// Optional DEIM gather (eq. grHDD with the exact potential), when dg.idx is
// set: with the field e_i just solved, g_F[k,i] = sum_r conj(U~[I_r,k]) w_r
// (q/m) e_i[j(x_{I_r,i})] over the d sampled rows, with the arithmetic of
// deim_gather_kernel operation by operation (the same bits).  The rows of U~
// at the sampled indices are loaded at the start, behind the partial sums.
struct DeimGatherArgs {
  const cplx* U;
  int N, n;
  const cplx* Z;
  const double* factor;
  double qm;
  const int* idx;
  const double* w;
  int d;
  cplx* gF;
  // optional fixed-point update of column i after the gather (counters set):
  // the arithmetic of dense_fp_update_kernel with linear_part on; counters[0]
  // loses one per column that stops, counters[1] gains the stalled ones,
  // counters[2] becomes the launch ordinal `iter` when a column was updated
  const cplx* C12;
  const cplx* Z0;
  cplx* Zeval;  // = Z, written for the columns that go on
  cplx* ZG;
  cplx* k;
  double* prev;
  int* active;
  double dt, tol, stall_tol;
  int fixed, iter;
  int* counters;
};

__global__ void __launch_bounds__(POISSON_THREADS) poisson_kernel(
    const double* __restrict__ part, int nrb, int p, int Nx, const double* __restrict__ qw,
    const double* __restrict__ h, const double* __restrict__ mw, const int* __restrict__ active,
    double* __restrict__ rho_out, double* __restrict__ phi_out, double* __restrict__ e_out,
    double* __restrict__ energy_out, const int* __restrict__ gate, DeimGatherArgs dg) {
  if (gate && gate[0] == 0) return;
  __shared__ double buf[POISSON_THREADS];
  __shared__ double rho_s[SYMROM_MAX_NX];   // the charge, later the field (DEIM gather)
  __shared__ cplx Ud[64 * SYMROM_MAX_NC];   // U~[I_r, k] at Ud[r * n + k]
  __shared__ cplx Zc[SYMROM_MAX_NC];        // column i of Z
  __shared__ cplx Cs[2 * 16 * 16];          // C12 when n <= 16
  __shared__ double Fw[64];
  const int i = blockIdx.x;
  if (active && !active[i]) return;
  const bool deim = dg.idx != nullptr;
  // everything the gather and the update read, loaded now, behind the
  // partial sums (the lanes that use a value in the tail load it here)
  const bool cs_lds = deim && dg.counters && dg.n <= 16;
  cplx kold = mk(0.0, 0.0), z0v = mk(0.0, 0.0);
  double wl = 0.0, prev_i = 0.0, fac_i = 1.0;
  if (deim) {
    const int t = threadIdx.x;
    fac_i = dg.factor[i];
    if (t < dg.d) {
      const int l = dg.idx[t];
      wl = dg.w[t];
      for (int k = 0; k < dg.n; ++k) Ud[t * dg.n + k] = dg.U[(size_t)k * dg.N + l];
    }
    if (t < dg.n) {
      Zc[t] = dg.Z[(size_t)i * dg.n + t];
      if (dg.counters) {
        kold = dg.k[(size_t)i * dg.n + t];
        z0v = dg.Z0[(size_t)i * dg.n + t];
      }
    }
    if (t == 0 && dg.counters) prev_i = dg.prev[i];
    if (cs_lds && t < 2 * dg.n * dg.n) Cs[t] = dg.C12[t];
  }
  const double hi = h[i];
  const double qwi = qw[i];
  // 1. sums of the unit weights over the nrb row-block partials
  //    part[(k * p + i) * Nx + j]: G = blockDim / Nx threads per node take
  //    every G-th block with all their loads in flight, then the G sums of a
  //    node are added in group order
  const int G = max(1, (int)blockDim.x / Nx);
  for (int t = threadIdx.x; t < G * Nx; t += blockDim.x) {
    const int j = t % Nx, g = t / Nx;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = g; k < nrb; k += 16 * G) {
      // loads at clamped indices (no branches), masked when added
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int kc = min(k + u * G, nrb - 1);
        v[u] = part[((size_t)kc * p + i) * Nx + j];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u & 3] += (k + u * G < nrb) ? v[u] : 0.0;
    }
    const double sg = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (G == 1)
      rho_s[j] = qwi * sg + hi;
    else
      buf[t] = sg;
  }
  __syncthreads();
  // the solve is one wavefront, nodes j0 .. j0 + per - 1 in lane `lane`
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  const int per = (Nx + 63) / 64;
  const int j0 = lane * per;
  double rho[POISSON_PER_LANE];
  double loc = 0.0;
#pragma unroll
  for (int q = 0; q < POISSON_PER_LANE; ++q) {
    const int j = j0 + q;
    rho[q] = 0.0;
    if (q < per && j < Nx) {
      if (G > 1) {
        double t2 = buf[j];
        for (int g = 1; g < G; ++g) t2 += buf[g * Nx + j];
        rho[q] = qwi * t2 + hi;
      } else {
        rho[q] = rho_s[j];
      }
    }
    loc += rho[q];
  }
  // 2. zero-mean charge, S_j = its inclusive prefix sums, e_j = mean(S) - S_j
  const double mean_rho = wave_sum64(loc) / Nx;
  double tot = 0.0;
#pragma unroll
  for (int q = 0; q < POISSON_PER_LANE; ++q)
    if (q < per && j0 + q < Nx) tot += rho[q] - mean_rho;
  double run = wave_exclusive_scan(tot);
  double S[POISSON_PER_LANE];
  double ssum = 0.0;
#pragma unroll
  for (int q = 0; q < POISSON_PER_LANE; ++q) {
    S[q] = 0.0;
    if (q < per && j0 + q < Nx) {
      run += rho[q] - mean_rho;
      S[q] = run;
      ssum += run;
    }
  }
  const double mean_S = wave_sum64(ssum) / Nx;
  double etot = 0.0;
#pragma unroll
  for (int q = 0; q < POISSON_PER_LANE; ++q) {
    S[q] = mean_S - S[q];  // e_j
    if (q < per && j0 + q < Nx) etot += S[q];
  }
  // 3. potential: Phi_j = h * sum_{k<j} e_k, then the zero-mean gauge
  double prun = wave_exclusive_scan(etot);
  double phi[POISSON_PER_LANE];
  double psum = 0.0;
#pragma unroll
  for (int q = 0; q < POISSON_PER_LANE; ++q) {
    phi[q] = 0.0;
    if (q < per && j0 + q < Nx) {
      phi[q] = hi * prun;
      prun += S[q];
      psum += phi[q];
    }
  }
  const double mean_phi = wave_sum64(psum) / Nx;
  double en = 0.0;
#pragma unroll
  for (int q = 0; q < POISSON_PER_LANE; ++q) {
    const int j = j0 + q;
    if (q < per && j < Nx) {
      const double ph = phi[q] - mean_phi;
      en += ph * rho[q];
      if (phi_out) phi_out[(size_t)i * Nx + j] = ph;
      if (rho_out) rho_out[(size_t)i * Nx + j] = rho[q];
      if (e_out) e_out[(size_t)i * Nx + j] = S[q];
    }
  }
  const double E = wave_sum64(en);
  if (lane == 0 && energy_out) energy_out[i] = E / (2.0 * mw[i]);
  if (!deim) return;
  // the field into LDS (the charge is in registers now), then the gather;
  // LDS accesses of this one wavefront take effect in program order
#pragma unroll
  for (int q = 0; q < POISSON_PER_LANE; ++q)
    if (q < per && j0 + q < Nx) rho_s[j0 + q] = S[q];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int n = dg.n;
  const cplx* zi = Zc;
  if (lane < dg.d) {
    double x = 0.0;
    for (int k = 0; k < n; ++k) {
      const cplx u = Ud[lane * n + k];
      x = fma(u.re, zi[k].re, x);
      x = fma(-u.im, zi[k].im, x);
    }
    int j;
    double th;
    cell_of(x, fac_i, Nx, j, th);
    Fw[lane] = wl * dg.qm * rho_s[j];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  cplx g = mk(0.0, 0.0);  // g_F[lane, i]
  for (int k = lane; k < n; k += 64) {
    cplx sk = mk(0.0, 0.0);
    for (int r = 0; r < dg.d; ++r) {
      const cplx u = Ud[r * n + k];
      sk.re = fma(u.re, Fw[r], sk.re);
      sk.im = fma(-u.im, Fw[r], sk.im);
    }
    dg.gF[(size_t)i * n + k] = sk;
    g = sk;
  }
  if (!dg.counters) return;
  // fixed-point update of column i (entries a = lane < n)
  const cplx* ze = zi;  // Z is the evaluation point of the iteration
  const cplx* C12 = cs_lds ? Cs : dg.C12;
  cplx knew = mk(0.0, 0.0);
  if (lane < n) {
    const int a = lane;
    cplx sl = mk(0.0, 0.0);
    for (int b = 0; b < n; ++b) {
      cfma(sl, C12[b * n + a], ze[b]);
      cfma(sl, cscale(cconj(C12[n * n + b * n + a]), -1.0), cconj(ze[b]));
    }
    g = cadd(g, cscale(sl, 0.5));
    knew = mk(g.im, -g.re);  // -i g
    const cplx dk = csub(knew, kold);
    buf[a] = cabs2(dk);
    buf[64 + a] = cabs2(knew);
    dg.k[(size_t)i * n + a] = knew;
    dg.ZG[(size_t)i * n + a] = ze[a];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane == 0) {
    double dn = 0.0, kn = 0.0;
    for (int a = 0; a < n; ++a) {
      dn += buf[a];
      kn += buf[64 + a];
    }
    bool done = false;
    if (!dg.fixed) {
      const double rel = (kn > 0.0) ? sqrt(dn) / sqrt(kn) : sqrt(dn);
      const bool conv = rel < dg.tol;
      const bool stall = !conv && rel >= prev_i && fmin(rel, prev_i) < dg.stall_tol;
      dg.prev[i] = rel;
      done = conv || stall;
      if (stall) {
        atomicAdd(&dg.counters[1], 1);
        atomicMax(reinterpret_cast<unsigned long long*>(dg.counters + 6),
                  (unsigned long long)__double_as_longlong(rel));
      }
    }
    if (done) {
      dg.active[i] = 0;
      atomicSub(&dg.counters[0], 1);
    }
    atomicMax(&dg.counters[2], dg.iter);
    Fw[0] = done ? 1.0 : 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (Fw[0] == 0.0 && lane < n) {
    const cplx z0 = z0v;
    dg.Zeval[(size_t)i * n + lane] =
        mk(z0.re + 0.5 * dg.dt * knew.re, z0.im + 0.5 * dg.dt * knew.im);
  }
}


// ---------------------------------------------------------------------------
// Full-order Stormer-Verlet in leapfrog form.  State (X_t, V_{t-1/2}).
//   kick:   V += ck * a(X),  a = -(q/m) e_{j(X)} from the current field
//   drift:  X += cd * V
//   deposit the new X (when `part` is non-null).
// One pass reads and writes X and V once: 32 bytes per particle-parameter.
// Grid (nrb, ntiles) as in deposit_x_kernel; LDS holds the field table and
// the histogram of the block's parameter tile.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(512) fom_push_kernel(
    double* __restrict__ X, double* __restrict__ V, int N, int p, int Nx, int pt, int rpb,
    const double* __restrict__ factor, const double* __restrict__ e, double qm, double ck,
    double cd, double* __restrict__ part) {
  extern __shared__ double smem[];
  double* et = smem;              // pt * Nx field table
  double* hist = smem + pt * Nx;  // pt * Nx theta sums per cell
  unsigned* cnt = reinterpret_cast<unsigned*>(smem + 2 * (size_t)pt * Nx);  // counts per cell
  const int rb = blockIdx.x;
  const int p0 = blockIdx.y * pt;
  const int np = min(pt, p - p0);
  for (int t = threadIdx.x; t < np * Nx; t += blockDim.x) {
    et[t] = e[(size_t)p0 * Nx + t];
    hist[t] = 0.0;
    cnt[t] = 0u;
  }
  __syncthreads();
  const int r0 = rb * rpb;
  const int r1 = min(N, r0 + rpb);
  for (int i = 0; i < np; ++i) {
    const double f = factor[p0 + i];
    double* Xi = X + (size_t)(p0 + i) * N;
    double* Vi = V + (size_t)(p0 + i) * N;
    const double* ei = et + i * Nx;
    double* hi = hist + i * Nx;
    unsigned* ci = cnt + i * Nx;
    for (int l = r0 + threadIdx.x; l < r1; l += blockDim.x) {
      double x = Xi[l];
      double v = Vi[l];
      int j;
      double th;
      cell_of(x, f, Nx, j, th);
      v = fma(ck, -qm * ei[j], v);
      x = fma(cd, v, x);
      Vi[l] = v;
      Xi[l] = x;
      if (part) {
        // count and theta per cell, as in deposit_rom_kernel
        cell_of(x, f, Nx, j, th);
        __hip_atomic_fetch_add(ci + j, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        lds_add(hi + j, th);
      }
    }
  }
  if (!part) return;
  __syncthreads();
  for (int t = threadIdx.x; t < np * Nx; t += blockDim.x) {
    const int i = t / Nx, j = t - i * Nx;
    const int jm = (j == 0) ? Nx - 1 : j - 1;
    part[((size_t)rb * p + p0) * Nx + t] = ((double)cnt[t] - hist[t]) + hist[i * Nx + jm];
  }
}

// V_out = V + c * a(X) without touching the state (full velocities from the
// staggered ones); also the kinetic energy is left to the caller.
__global__ void fom_velocity_kernel(const double* __restrict__ X, const double* __restrict__ V,
                                    int N, int p, int Nx, const double* __restrict__ factor,
                                    const double* __restrict__ e, double qm, double c,
                                    double* __restrict__ Vout) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t tot = (size_t)N * p;
  if (t >= tot) return;
  int i = (int)(t / N);
  int j;
  double th;
  cell_of(X[t], factor[i], Nx, j, th);
  Vout[t] = fma(c, -qm * e[(size_t)i * Nx + j], V[t]);
}

// Cell index of every particle (int32, N x p).
__global__ void cells_kernel(const double* __restrict__ X, int N, int p, int Nx,
                             const double* __restrict__ factor, int* __restrict__ cells) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t tot = (size_t)N * p;
  if (t >= tot) return;
  int i = (int)(t / N);
  int j;
  double th;
  cell_of(X[t], factor[i], Nx, j, th);
  cells[t] = j;
}

// Cell index and scaled position s = x N_x / L of every (particle,
// parameter) of the reduced model, with the position arithmetic of
// deposit_rom_kernel operation by operation (masked register row of U~,
// even and odd columns summed apart, then added): the cells the fused
// kernels use, for checking them against an independent reconstruction.
template <int NC>
__global__ void __launch_bounds__(256) rom_cells_kernel(const cplx* __restrict__ U, int N, int n,
                                                        const cplx* __restrict__ Z, int p, int Nx,
                                                        const double* __restrict__ factor,
                                                        int* __restrict__ cells,
                                                        double* __restrict__ sv) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= N) return;
  cplx u[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const cplx v = U[(size_t)min(k, n - 1) * N + l];
    const double m = (k < n) ? 1.0 : 0.0;
    u[k] = mk(v.re * m, v.im * m);
  }
  for (int i = 0; i < p; ++i) {
    cplx z[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const cplx a = Z[(size_t)i * n + min(k, n - 1)];
      z[k] = (k < n) ? a : mk(0.0, 0.0);
    }
    double x0 = 0.0, x1 = 0.0;
#pragma unroll
    for (int k = 0; k < NC; k += 2) {
      x0 = fma(u[k].re, z[k].re, x0);
      x0 = fma(-u[k].im, z[k].im, x0);
      if (k + 1 < NC) {
        x1 = fma(u[k + 1].re, z[k + 1].re, x1);
        x1 = fma(-u[k + 1].im, z[k + 1].im, x1);
      }
    }
    const double x = x0 + x1;
    int j;
    double th;
    cell_of(x, factor[i], Nx, j, th);
    cells[(size_t)i * N + l] = j;
    if (sv) sv[(size_t)i * N + l] = x * factor[i];
  }
}

void launch_rom_cells(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                      const double* factor, int* cells, double* sv) {
  const int nc = (n <= 16) ? nc_even(n) : 32;
  dim3 grid((N + 255) / 256);
#define RCL(NCV)                                                                              \
  hipLaunchKernelGGL(rom_cells_kernel<NCV>, grid, dim3(256), 0, s, U, N, n, Z, p, Nx, factor, \
                     cells, sv)
  switch (nc) {
    case 4: RCL(4); break;
    case 5: RCL(5); break;
    case 6: RCL(6); break;
    case 7: RCL(7); break;
    case 8: RCL(8); break;
    case 12: RCL(12); break;
    case 16: RCL(16); break;
    default: RCL(32); break;
  }
#undef RCL
}

// Per-parameter sum of squares of the columns of an N x p matrix, times s:
// grid (p, chunks) partial sums, combined in order by the second kernel.
#define CSQ_CHUNKS 32
__global__ void __launch_bounds__(256) colsumsq_part_kernel(const double* __restrict__ A, int N,
                                                            double* __restrict__ part) {
  __shared__ double red[8];
  const int i = blockIdx.x, c = blockIdx.y;
  const double* a = A + (size_t)i * N;
  const int per = (N + CSQ_CHUNKS - 1) / CSQ_CHUNKS;
  const int l0 = c * per, l1 = min(N, l0 + per);
  double acc = 0.0;
  for (int l = l0 + threadIdx.x; l < l1; l += blockDim.x) acc = fma(a[l], a[l], acc);
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[(size_t)i * CSQ_CHUNKS + c] = acc;
}
__global__ void colsumsq_fin_kernel(const double* __restrict__ part, int p, double s,
                                    double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p) return;
  double t = 0.0;
  for (int c = 0; c < CSQ_CHUNKS; ++c) t += part[(size_t)i * CSQ_CHUNKS + c];
  out[i] = s * t;
}

// out[i] += in[i]
__global__ void vec_add_kernel(double* __restrict__ out, const double* __restrict__ in, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] += in[t];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
void launch_deposit_x(hipStream_t s, const double* X, int N, int p, int Nx, const PicGeom& g,
                      const double* factor, double* part) {
  ALLOW_BIG_LDS(deposit_x_kernel);
  dim3 grid(g.nrb, (p + g.pt - 1) / g.pt);
  size_t sh = (size_t)g.pt * Nx * sizeof(double);
  hipLaunchKernelGGL(deposit_x_kernel, grid, dim3(512), sh, s, X, N, p, Nx, g.pt, g.rpb, factor,
                     part);
}

void launch_deposit_rom(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                        const PicGeom& g, const double* factor, const int* active, double* part,
                        const int* gate, int* fold, int det) {
  int nc = (n <= 16) ? nc_even(n) : 32;
  if (n <= 16) {
    // positions on the matrix cores, tiles of deposit_tile_params(Nx)
    // parameters (the row blocks of g)
    const int pte = deposit_tile_params(Nx);
    dim3 gridm(g.nrb, (p + pte - 1) / pte);
    const size_t shm = (size_t)pte * Nx * (sizeof(double) + sizeof(unsigned));
#define DEPM(NCV)                                                                                 \
  ALLOW_BIG_LDS(deposit_rom_mfma_kernel<NCV>);                                                   \
  hipLaunchKernelGGL(deposit_rom_mfma_kernel<NCV>, gridm, dim3(1024), shm, s, U, N, n, Z, p, Nx,  \
                     pte, g.rpb, factor, active, part, gate, fold, det)
    switch (nc) {
      case 4: DEPM(4); break;
      case 5: DEPM(5); break;
      case 6: DEPM(6); break;
      case 7: DEPM(7); break;
      case 8: DEPM(8); break;
      case 12: DEPM(12); break;
      default: DEPM(16); break;
    }
#undef DEPM
    return;
  }
  dim3 grid(g.nrb, (p + g.pt - 1) / g.pt);
  size_t sh = (size_t)g.pt * Nx * (sizeof(double) + sizeof(unsigned));
#define DEP(NCV)                                                                              \
  ALLOW_BIG_LDS(deposit_rom_kernel<NCV>);                                                    \
  hipLaunchKernelGGL(deposit_rom_kernel<NCV>, grid, dim3(deposit_rom_threads<NCV>()), sh, s, U, \
                     N, n, Z, p, Nx, g.pt, g.rpb, factor, active, part, gate, fold, det)
  switch (nc) {
    case 4: DEP(4); break;
    case 5: DEP(5); break;
    case 6: DEP(6); break;
    case 7: DEP(7); break;
    case 8: DEP(8); break;
    case 12: DEP(12); break;
    case 16: DEP(16); break;
    default: DEP(32); break;
  }
#undef DEP
}

void launch_poisson(hipStream_t s, const double* part, int nrb, int p, int Nx, const double* qw,
                    const double* h, const double* mw, const int* active, double* rho,
                    double* phi, double* e, double* energy, const int* gate) {
  // one block per parameter sums its row-block partials and solves
  DeimGatherArgs dg{};
  hipLaunchKernelGGL(poisson_kernel, dim3(p), dim3(POISSON_THREADS), 0, s, part, nrb, p, Nx, qw, h,
                     mw, active, rho, phi, e, energy, gate, dg);
}

void launch_poisson_deim(hipStream_t s, const double* part, int nrb, int p, int Nx,
                         const double* qw, const double* h, const double* mw, int* active,
                         double* rho, double* phi, double* e, double* energy, const int* gate,
                         const cplx* U, int N, int n, cplx* Z, const double* factor, double qm,
                         const int* idx, const double* w, int d, cplx* gF, const cplx* C12,
                         const cplx* Z0, cplx* ZG, cplx* k, double* prev, double dt, double tol,
                         double stall_tol, int fixed, int iter, int* counters) {
  DeimGatherArgs dg{U,   N,  n,    Z,      factor, qm,  idx,       w,     d,    gF,      C12,
                    Z0,  Z,  ZG,   k,      prev,   active, dt, tol, stall_tol, fixed, iter, counters};
  hipLaunchKernelGGL(poisson_kernel, dim3(p), dim3(POISSON_THREADS), 0, s, part, nrb, p, Nx, qw, h,
                     mw, active, rho, phi, e, energy, gate, dg);
}

void launch_fom_push(hipStream_t s, double* X, double* V, int N, int p, int Nx, const PicGeom& g,
                     const double* factor, const double* e, double qm, double ck, double cd,
                     double* part) {
  dim3 grid(g.nrb, (p + g.pt - 1) / g.pt);
  size_t sh = (size_t)g.pt * Nx * (2 * sizeof(double) + sizeof(unsigned));
  ALLOW_BIG_LDS(fom_push_kernel);
  hipLaunchKernelGGL(fom_push_kernel, grid, dim3(512), sh, s, X, V, N, p, Nx, g.pt, g.rpb, factor,
                     e, qm, ck, cd, part);
}

void launch_fom_velocity(hipStream_t s, const double* X, const double* V, int N, int p, int Nx,
                         const double* factor, const double* e, double qm, double c,
                         double* Vout) {
  size_t tot = (size_t)N * p;
  hipLaunchKernelGGL(fom_velocity_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X,
                     V, N, p, Nx, factor, e, qm, c, Vout);
}

void launch_cells(hipStream_t s, const double* X, int N, int p, int Nx, const double* factor,
                  int* cells) {
  size_t tot = (size_t)N * p;
  hipLaunchKernelGGL(cells_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, N, p,
                     Nx, factor, cells);
}

void launch_colsumsq(hipStream_t s, const double* A, int N, int p, double sc, double* out,
                     double* scratch) {
  hipLaunchKernelGGL(colsumsq_part_kernel, dim3(p, CSQ_CHUNKS), dim3(256), 0, s, A, N, scratch);
  hipLaunchKernelGGL(colsumsq_fin_kernel, dim3((p + 255) / 256), dim3(256), 0, s, scratch, p, sc,
                     out);
}

void launch_vec_add(hipStream_t s, double* out, const double* in, int n) {
  hipLaunchKernelGGL(vec_add_kernel, dim3((n + 255) / 256), dim3(256), 0, s, out, in, n);
}
