// Shared device helpers for the symrom HIP library (gfx950).
//
// Storage conventions inside the library
//   * complex basis U~ = A + iB (N x n) is stored column-major with leading
//     dimension N, each element an interleaved (re, im) pair of doubles;
//   * complex coefficients Z~ = Z_q + i Z_p (n x p) column-major, ld = n;
//   * grids (rho, Phi, e) are p x Nx row-major: row i is parameter i.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct cplx {
  double re, im;
};

__host__ __device__ inline cplx mk(double r, double i) { return cplx{r, i}; }
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cplx csub(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cplx cmul(cplx a, cplx b) {
  return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
__host__ __device__ inline cplx cmulc(cplx a, cplx b) {
  return cplx{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__host__ __device__ inline cplx cconj(cplx a) { return cplx{a.re, -a.im}; }
__host__ __device__ inline cplx cscale(cplx a, double s) { return cplx{a.re * s, a.im * s}; }
// acc += a * b
__host__ __device__ inline void cfma(cplx& acc, cplx a, cplx b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
__host__ __device__ inline void cfmac(cplx& acc, cplx a, cplx b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
__host__ __device__ inline double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }

// Particle-to-cell lookup of the periodic P1 mesh.  s = x * (Nx / L) with the
// factor formed once in FP64 on the host; c = floor(s); theta = s - c (exact);
// node j = c mod Nx (Euclidean).  A particle on a node takes the cell to its
// right.  Exact for unwrapped positions with |s| < 2^52.  Beyond that, and for
// a non-finite position (a diverged state), the cell is still some j in
// [0, Nx), so that no lookup or deposit leaves its table.  Branch-free, so
// that the cells of several particles of a thread interleave.
__device__ inline void cell_of(double x, double factor, int Nx, int& j, double& theta) {
  const double s = x * factor;
  const double c = floor(s);
  theta = s - c;
  // Euclidean c mod Nx in exact double arithmetic (c and q*Nx are integers
  // below 2^53); the quotient estimate is corrected by at most one.
  const double fNx = (double)Nx;
  const double q = floor(c * (1.0 / fNx));
  double r = fma(-q, fNx, c);
  r = (r < 0.0) ? r + fNx : r;
  r = (r >= fNx) ? r - fNx : r;
  // (no effect in the exact range; fmax takes 0 for a NaN)
  r = fmin(fmax(r, 0.0), fNx - 1.0);
  j = (int)r;
}

// ---------------------------------------------------------------------------
// Particle positions on the FP64 matrix cores (v_mfma_f64_16x16x4f64: a
// wavefront multiplies a 16 x 4 tile A by a 4 x 16 tile B into a 16 x 16
// accumulator; A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, and lane
// l holds D[4 v + l / 16][l % 16] in item v).  In real form with K = 2 NC,
// X = a b with a = [Re U~ | -Im U~] (one row per particle) and b = [Re Z~;
// Im Z~], for 16 particle rows against 16 parameters: lane li + 16 lk holds
// a[row + li][4 ks + lk] and b[4 ks + lk][parameter li] for step ks, and ends
// with the positions of rows 4 v + lk of its parameter li.  Every kernel
// that deposits or gathers at these positions forms them with this code,
// so that a particle lands in the same cell in each.
// ---------------------------------------------------------------------------
typedef double mf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mf4 mfma_f64_step(double a, double b, mf4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Entries of a: the column, component (re or im) and sign (+1, -1 for
// -Im, 0 past n or past 2 NC) of entry q are fixed per lane, so they are set
// up once; a zero entry reads column 0.
template <int KS>
struct PosRows {
  const double* ptr[KS];
  double sgn[KS];
  __device__ __forceinline__ void setup(const cplx* __restrict__ U, int N, int n, int NC,
                                        int lk) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int q = 4 * ks + lk;
      const int col = (q < NC) ? q : q - NC;
      const bool ok = q < 2 * NC && col < n;
      ptr[ks] = reinterpret_cast<const double*>(U + (size_t)(ok ? col : 0) * N) + (q < NC ? 0 : 1);
      sgn[ks] = ok ? (q < NC ? 1.0 : -1.0) : 0.0;
    }
  }
  // a[ks] for particle row `row` (this lane's row of the tile)
  __device__ __forceinline__ void load(int row, double* a) const {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a[ks] = sgn[ks] * ptr[ks][2 * (size_t)row];
  }
};

// Entries of b for parameter c (zero past n, or everywhere when !on)
template <int KS>
__device__ __forceinline__ void pos_coefs(const cplx* __restrict__ Z, int n, int NC, int c,
                                          bool on, int lk, double* bz) {
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int q = 4 * ks + lk;
    double v = 0.0;
    if (q < NC) {
      if (q < n) v = Z[(size_t)c * n + q].re;
    } else if (q - NC < n && q - NC < NC) {
      v = Z[(size_t)c * n + (q - NC)].im;
    }
    bz[ks] = on ? v : 0.0;
  }
}

// X for the tile: the KS steps in order from zero
template <int KS>
__device__ __forceinline__ mf4 pos_tile(const double* a, const double* bz) {
  mf4 X = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) X = mfma_f64_step(a[ks], bz[ks], X);
  return X;
}

// LDS FP64 atomic add (hardware ds_add_f64 on gfx950)
__device__ inline void lds_add(double* addr, double v) {
  __hip_atomic_fetch_add(addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Block-wide sum of one double; every thread receives the result.
// `red` is an LDS scratch of at least blockDim.x/64 doubles.
__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  __syncthreads();
  return t;
}

// Allow a kernel to use the full 160 KB of LDS of a gfx950 workgroup for its
// dynamic allocation (the cap is reduced by the kernel's static LDS).  The
// attribute call's error state is consumed here so that it never surfaces in
// a later launch check.
template <class K>
inline void allow_big_lds(K kern) {
  hipFuncAttributes a;
  if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(kern)) == hipSuccess) {
    int dyn = 160 * 1024 - (int)a.sharedSizeBytes;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
  }
  (void)hipGetLastError();
}
#define ALLOW_BIG_LDS(kern)   \
  do {                        \
    static bool done_ = false; \
    if (!done_) {             \
      allow_big_lds(kern);    \
      done_ = true;           \
    }                         \
  } while (0)

#define SYMROM_MAX_NC 32    // complex reduced columns held in registers (2n <= 64)
#define SYMROM_MAX_NX 1024  // grid nodes handled by the Poisson kernel

// One 64-bit DPP move (two 32-bit moves; zero where the source lane is out
// of range or its row is masked off).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Butterfly partners inside aligned groups of up to 16 lanes: lane i ^ 1
// and i ^ 2 (quad permutations), then the mirror images inside halves of 8
// and rows of 16, which pair every lane with one in the other half.
// Combining with a commutative operation leaves the same bits in every lane
// of the group.
template <int LEVEL>
__device__ __forceinline__ double bfly64(double v) {
  if (LEVEL == 0) return dpp64<0xB1, 0xf>(v);    // quad_perm [1,0,3,2]
  if (LEVEL == 1) return dpp64<0x4E, 0xf>(v);    // quad_perm [2,3,0,1]
  if (LEVEL == 2) return dpp64<0x141, 0xf>(v);   // row_half_mirror
  return dpp64<0x140, 0xf>(v);                   // row_mirror
}

// the same butterfly for 32-bit integers
template <int LEVEL>
__device__ __forceinline__ int bfly32(int v) {
  constexpr int CTRL = (LEVEL == 0) ? 0xB1 : (LEVEL == 1) ? 0x4E : (LEVEL == 2) ? 0x141 : 0x140;
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true);
}

// value of v in lane `lane` (uniform), as a scalar
__device__ __forceinline__ double rdlane64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __hiloint2double(hi, lo);
}

// sum over the 64 lanes of a wavefront, the same bits in every lane: row
// butterflies, then the four row sums added in a fixed order
__device__ __forceinline__ double wave_sum64(double v) {
  v += bfly64<0>(v);
  v += bfly64<1>(v);
  v += bfly64<2>(v);
  v += bfly64<3>(v);
  return (rdlane64(v, 0) + rdlane64(v, 16)) + (rdlane64(v, 32) + rdlane64(v, 48));
}
