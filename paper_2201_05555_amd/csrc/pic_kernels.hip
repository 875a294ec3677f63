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
// One thread per particle row holds its n complex basis entries in
// registers; the coefficient tile is broadcast from LDS.  Columns whose
// `active` flag is 0 are skipped (frozen fixed-point columns).
// ---------------------------------------------------------------------------
template <int NC>
__global__ void __launch_bounds__(512) deposit_rom_kernel(
    const cplx* __restrict__ U, int N, int n, const cplx* __restrict__ Z, int p, int Nx, int pt,
    int rpb, const double* __restrict__ factor, const int* __restrict__ active,
    double* __restrict__ part, const int* __restrict__ gate) {
  if (gate && gate[0] == 0) return;
  // parameters in flight per thread (independent chains), within registers
  constexpr int ILP = (NC <= 8) ? 4 : (NC <= 16) ? 2 : 1;
  extern __shared__ double smem[];
  double* hist = smem;                                  // pt * Nx
  cplx* Zs = reinterpret_cast<cplx*>(smem + pt * Nx);   // pt * NC
  double* fs = reinterpret_cast<double*>(Zs + pt * NC);  // pt factors
  int* act = reinterpret_cast<int*>(fs + pt);            // pt flags
  const int rb = blockIdx.x;
  const int p0 = blockIdx.y * pt;
  const int np = min(pt, p - p0);
  for (int t = threadIdx.x; t < np * Nx; t += blockDim.x) hist[t] = 0.0;
  for (int t = threadIdx.x; t < np * NC; t += blockDim.x) {
    int i = t / NC, k = t % NC;
    Zs[t] = (k < n) ? Z[(size_t)(p0 + i) * n + k] : mk(0.0, 0.0);
  }
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    fs[i] = factor[p0 + i];
    act[i] = active ? active[p0 + i] : 1;
  }
  __syncthreads();
  const int r0 = rb * rpb;
  const int r1 = min(N, r0 + rpb);
  for (int l = r0 + threadIdx.x; l < r1; l += blockDim.x) {
    cplx u[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) u[k] = (k < n) ? U[(size_t)k * N + l] : mk(0.0, 0.0);
    // ILP parameters at a time: their position sums, cell lookups and
    // histogram updates are independent and interleave
    for (int i0 = 0; i0 < np; i0 += ILP) {
      double x0[ILP], x1[ILP];
#pragma unroll
      for (int q = 0; q < ILP; ++q) {
        x0[q] = 0.0;
        x1[q] = 0.0;
      }
#pragma unroll
      for (int q = 0; q < ILP; ++q) {
        const cplx* zi = Zs + min(i0 + q, np - 1) * NC;
#pragma unroll
        for (int k = 0; k < NC; k += 2) {
          x0[q] = fma(u[k].re, zi[k].re, x0[q]);
          x0[q] = fma(-u[k].im, zi[k].im, x0[q]);
          x1[q] = fma(u[k + 1].re, zi[k + 1].re, x1[q]);
          x1[q] = fma(-u[k + 1].im, zi[k + 1].im, x1[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < ILP; ++q) {
        const int i = i0 + q;
        int j;
        double th;
        cell_of(x0[q] + x1[q], fs[min(i, np - 1)], Nx, j, th);
        if (i < np && act[i]) {
          const int j1 = (j + 1 == Nx) ? 0 : j + 1;
          lds_add(hist + i * Nx + j, 1.0 - th);
          lds_add(hist + i * Nx + j1, th);
        }
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < np * Nx; t += blockDim.x) {
    int i = t / Nx;
    if (!act[i]) continue;
    part[((size_t)rb * p + p0) * Nx + t] = hist[t];
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
__device__ inline double block_exclusive_scan(double v, double* buf) {
  // Hillis-Steele inclusive scan over blockDim.x thread values, then shift
  const int t = threadIdx.x;
  buf[t] = v;
  __syncthreads();
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {
    double add = (t >= o) ? buf[t - o] : 0.0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  double incl = buf[t];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(256) poisson_kernel(
    const double* __restrict__ part, int nrb, int p, int Nx, const double* __restrict__ qw,
    const double* __restrict__ h, const double* __restrict__ mw, const int* __restrict__ active,
    double* __restrict__ rho_out, double* __restrict__ phi_out, double* __restrict__ e_out,
    double* __restrict__ energy_out, const int* __restrict__ gate) {
  if (gate && gate[0] == 0) return;
  __shared__ double buf[256];
  __shared__ double red[8];
  __shared__ double rho_s[SYMROM_MAX_NX];
  __shared__ double e_s[SYMROM_MAX_NX];
  const int i = blockIdx.x;
  if (active && !active[i]) return;
  const int per = (Nx + blockDim.x - 1) / blockDim.x;  // nodes per thread (contiguous)
  const int j0 = threadIdx.x * per;
  const double hi = h[i];
  const double qwi = qw[i];
  // 1. sums of the unit weights over the nrb row-block partials
  //    part[(k * p + i) * Nx + j]: G threads per node take every G-th block,
  //    two chains each, combined in a fixed order
  {
    const int G = (Nx <= 64) ? 4 : (Nx <= 128) ? 2 : 1;
    for (int t = threadIdx.x; t < G * Nx; t += blockDim.x) {
      const int j = t % Nx, g = t / Nx;
      // eight partials in flight per thread, summed in block order
      double acc8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc8[u] = 0.0;
      int k = g;
      for (; k + 7 * G < nrb; k += 8 * G) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc8[u] += part[((size_t)(k + u * G) * p + i) * Nx + j];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int kq = k + u * G;
        if (kq < nrb) acc8[u] += part[((size_t)kq * p + i) * Nx + j];
      }
      const double s01 = ((acc8[0] + acc8[1]) + (acc8[2] + acc8[3])) +
                         ((acc8[4] + acc8[5]) + (acc8[6] + acc8[7]));
      if (G == 1)
        rho_s[j] = qwi * s01 + hi;
      else
        buf[g * Nx + j] = s01;
    }
    __syncthreads();
    if (G > 1) {
      for (int j = threadIdx.x; j < Nx; j += blockDim.x) {
        double t2 = buf[j];
        for (int g = 1; g < G; ++g) t2 += buf[g * Nx + j];
        rho_s[j] = qwi * t2 + hi;
      }
      __syncthreads();
    }
  }
  // 2. zero-mean charge and its prefix sums
  double loc = 0.0;
  for (int q = 0; q < per; ++q)
    if (j0 + q < Nx) loc += rho_s[j0 + q];
  const double mean_rho = block_sum(loc, red) / Nx;
  double tot = 0.0;
  for (int q = 0; q < per; ++q)
    if (j0 + q < Nx) tot += rho_s[j0 + q] - mean_rho;
  double run = block_exclusive_scan(tot, buf);
  double ssum = 0.0;
  for (int q = 0; q < per; ++q) {
    int j = j0 + q;
    if (j < Nx) {
      run += rho_s[j] - mean_rho;
      e_s[j] = run;  // S_j for now
      ssum += run;
    }
  }
  const double mean_S = block_sum(ssum, red) / Nx;
  double etot = 0.0;
  for (int q = 0; q < per; ++q) {
    int j = j0 + q;
    if (j < Nx) {
      e_s[j] = mean_S - e_s[j];
      etot += e_s[j];
    }
  }
  // 3. potential: Phi_j = h * sum_{k<j} e_k, then the zero-mean gauge
  double prun = block_exclusive_scan(etot, buf);
  double phi_loc[8];
  double psum = 0.0;
  for (int q = 0; q < per; ++q) {
    int j = j0 + q;
    if (j < Nx) {
      phi_loc[q] = hi * prun;
      prun += e_s[j];
      psum += phi_loc[q];
    }
  }
  const double mean_phi = block_sum(psum, red) / Nx;
  double en = 0.0;
  for (int q = 0; q < per; ++q) {
    int j = j0 + q;
    if (j < Nx) {
      double ph = phi_loc[q] - mean_phi;
      en += ph * rho_s[j];
      if (phi_out) phi_out[(size_t)i * Nx + j] = ph;
      if (rho_out) rho_out[(size_t)i * Nx + j] = rho_s[j];
      if (e_out) e_out[(size_t)i * Nx + j] = e_s[j];
    }
  }
  const double E = block_sum(en, red);
  if (threadIdx.x == 0 && energy_out) energy_out[i] = E / (2.0 * mw[i]);
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
  double* et = smem;            // pt * Nx field table
  double* hist = smem + pt * Nx;  // pt * Nx
  const int rb = blockIdx.x;
  const int p0 = blockIdx.y * pt;
  const int np = min(pt, p - p0);
  for (int t = threadIdx.x; t < np * Nx; t += blockDim.x) {
    et[t] = e[(size_t)p0 * Nx + t];
    hist[t] = 0.0;
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
        cell_of(x, f, Nx, j, th);
        int j1 = (j + 1 == Nx) ? 0 : j + 1;
        lds_add(hi + j, 1.0 - th);
        lds_add(hi + j1, th);
      }
    }
  }
  if (!part) return;
  __syncthreads();
  for (int t = threadIdx.x; t < np * Nx; t += blockDim.x)
    part[((size_t)rb * p + p0) * Nx + t] = hist[t];
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
                        const int* gate) {
  dim3 grid(g.nrb, (p + g.pt - 1) / g.pt);
  int nc = (n <= 16) ? nc_even(n) : 32;
  size_t sh = (size_t)g.pt * Nx * sizeof(double) + (size_t)g.pt * nc * sizeof(cplx) +
              (size_t)g.pt * (sizeof(double) + sizeof(int));
#define DEP(NCV)                                                                              \
  ALLOW_BIG_LDS(deposit_rom_kernel<NCV>);                                                    \
  hipLaunchKernelGGL(deposit_rom_kernel<NCV>, grid, dim3(512), sh, s, U, N, n, Z, p, Nx, g.pt, \
                     g.rpb, factor, active, part, gate)
  switch (nc) {
    case 4: DEP(4); break;
    case 6: DEP(6); break;
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
  hipLaunchKernelGGL(poisson_kernel, dim3(p), dim3(256), 0, s, part, nrb, p, Nx, qw, h, mw, active,
                     rho, phi, e, energy, gate);
}

void launch_fom_push(hipStream_t s, double* X, double* V, int N, int p, int Nx, const PicGeom& g,
                     const double* factor, const double* e, double qm, double ck, double cd,
                     double* part) {
  dim3 grid(g.nrb, (p + g.pt - 1) / g.pt);
  size_t sh = 2 * (size_t)g.pt * Nx * sizeof(double);
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
