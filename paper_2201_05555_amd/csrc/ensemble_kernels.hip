// Kernels for large ensembles (many parameters p): the p x p Gram of an
// N x p matrix assembled from 64-column blocks, the leading eigenvectors of
// a p x p Hermitian matrix by subspace iteration (products with the matrix,
// classical Gram-Schmidt applied twice), and the device-side loading of the
// initial ensemble from its parameters and shared uniforms.
#include "common.h"
#include "kernels.h"

// G[a0 + i, b0 + j] = blk[i, j] and, off the diagonal block,
// G[b0 + j, a0 + i] = conj(blk[i, j]) (blk: ac x bc column-major, G: ld p).
__global__ void scatter_block_kernel(const cplx* __restrict__ blk, int ac, int bc,
                                     cplx* __restrict__ G, int p, int a0, int b0) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ac * bc) return;
  const int i = t % ac, j = t / ac;
  const cplx v = blk[t];
  G[(size_t)(b0 + j) * p + a0 + i] = v;
  if (a0 != b0) G[(size_t)(a0 + i) * p + b0 + j] = cconj(v);
}

void launch_scatter_block(hipStream_t s, const cplx* blk, int ac, int bc, cplx* G, int p, int a0,
                          int b0) {
  hipLaunchKernelGGL(scatter_block_kernel, dim3((ac * bc + 255) / 256), dim3(256), 0, s, blk, ac,
                     bc, G, p, a0, b0);
}

// W = A V for A p x p (column-major, ld p) and V p x m (ld p): one output
// entry per thread, the lanes of a wavefront on consecutive rows (coalesced
// columns of A, one entry of V per wavefront and step).
__global__ void __launch_bounds__(256) herm_mm_kernel(const cplx* __restrict__ A,
                                                      const cplx* __restrict__ V, int p, int m,
                                                      cplx* __restrict__ W) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= p * m) return;
  const int r = t % p, c = t / p;
  const cplx* vc = V + (size_t)c * p;
  cplx acc = mk(0.0, 0.0);
  for (int q = 0; q < p; ++q) cfma(acc, A[(size_t)q * p + r], vc[q]);
  W[t] = acc;
}

void launch_herm_mm(hipStream_t s, const cplx* A, const cplx* V, int p, int m, cplx* W) {
  hipLaunchKernelGGL(herm_mm_kernel, dim3((p * m + 255) / 256), dim3(256), 0, s, A, V, p, m, W);
}

// Orthonormal columns of W (p x m, ld p) by classical Gram-Schmidt applied
// twice per column, in one workgroup: the projections of column j on the
// previous ones are summed one wavefront per previous column, then removed
// from all entries at once.  A column whose norm drops below 1e-13 of its
// norm before the projections (it lies in the span of the previous ones) is
// replaced by a fixed pseudo-random vector and orthogonalised again, so the
// result always has m orthonormal columns (m <= 64).
__global__ void __launch_bounds__(256) cgs2_kernel(cplx* __restrict__ W, int p, int m) {
  __shared__ cplx dots[64];
  __shared__ double red[4];
  __shared__ double nrm0, nrm1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int j = 0; j < m; ++j) {
    cplx* wj = W + (size_t)j * p;
    for (int attempt = 0; attempt < 3; ++attempt) {
      // norm before the projections
      double s0 = 0.0;
      for (int l = tid; l < p; l += 256) s0 += cabs2(wj[l]);
      for (int o = 32; o > 0; o >>= 1) s0 += __shfl_xor(s0, o, 64);
      if (lane == 0) red[wv] = s0;
      __syncthreads();
      if (tid == 0) nrm0 = sqrt(((red[0] + red[1]) + red[2]) + red[3]);
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass) {
        for (int i = wv; i < j; i += 4) {
          const cplx* wi = W + (size_t)i * p;
          cplx d = mk(0.0, 0.0);
          for (int l = lane; l < p; l += 64) cfmac(d, wi[l], wj[l]);
          for (int o = 32; o > 0; o >>= 1) {
            d.re += __shfl_xor(d.re, o, 64);
            d.im += __shfl_xor(d.im, o, 64);
          }
          if (lane == 0) dots[i] = d;
        }
        __syncthreads();
        for (int l = tid; l < p; l += 256) {
          cplx v = wj[l];
          for (int i = 0; i < j; ++i) v = csub(v, cmul(dots[i], W[(size_t)i * p + l]));
          wj[l] = v;
        }
        __syncthreads();
      }
      double s1 = 0.0;
      for (int l = tid; l < p; l += 256) s1 += cabs2(wj[l]);
      for (int o = 32; o > 0; o >>= 1) s1 += __shfl_xor(s1, o, 64);
      if (lane == 0) red[wv] = s1;
      __syncthreads();
      if (tid == 0) nrm1 = sqrt(((red[0] + red[1]) + red[2]) + red[3]);
      __syncthreads();
      const double a = nrm1, b = nrm0;
      if (a > 1e-13 * b && a > 1e-300) {
        for (int l = tid; l < p; l += 256) wj[l] = cscale(wj[l], 1.0 / a);
        __syncthreads();
        break;
      }
      // dependent column: a fixed pseudo-random replacement, then again
      for (int l = tid; l < p; l += 256) {
        unsigned x = (unsigned)(l * 2654435761u) ^ (unsigned)((j + 1) * 40503u + attempt * 977u);
        x ^= x >> 13;
        x *= 0x5bd1e995u;
        x ^= x >> 15;
        wj[l] = mk((double)(x & 0xffff) / 65536.0 - 0.5, (double)(x >> 16) / 65536.0 - 0.5);
      }
      __syncthreads();
    }
  }
}

void launch_cgs2(hipStream_t s, cplx* W, int p, int m) {
  hipLaunchKernelGGL(cgs2_kernel, dim3(1), dim3(256), 0, s, W, p, m);
}

// ---------------------------------------------------------------------------
// Initial ensemble from its parameters (Sec. 6.1 loading of the perturbed
// Maxwellian f0(x, v) = f_v(v) (1 + alpha cos kx) on [0, 2 pi / k) x
// [-10, 10]): for particle l and parameter i, with uniforms u_x[l], u_v[l]
// shared by every parameter,
//   x = F_x^{-1}(u_x),  F_x(x) = (x + (alpha / k) sin kx) / L   (Newton,
//       iterates kept in [0, L], stop when the step is below 1e-15 L);
//   v = F_v^{-1}(lo + u_v (hi - lo)), lo, hi = F_v(-10), F_v(10), with F_v
//       the CDF of N(0, sigma) (family 0: Landau; closed form through the
//       inverse normal CDF) or of (N(-v0, sigma) + N(+v0, sigma)) / 2
//       (family 1: two-stream; start from the nearer beam, then Newton kept
//       inside a shrinking bracket, bisection where a step leaves it).
// eta: device, p x 4 row-major (alpha, k, v0, sigma).  Outputs X, V (N x p,
// column-major, nullable) and/or C = X + i V (nullable).
// ---------------------------------------------------------------------------
__device__ inline double std_cdf(double z) { return 0.5 * erfc(-z * 0.70710678118654752440); }

__device__ inline double mix_cdf(double v, double v0, double sg) {
  return 0.5 * (std_cdf((v - v0) / sg) + std_cdf((v + v0) / sg));
}

__device__ inline double mix_pdf(double v, double v0, double sg) {
  const double a = (v - v0) / sg, b = (v + v0) / sg;
  return 0.5 * (exp(-0.5 * a * a) + exp(-0.5 * b * b)) / (sg * 2.50662827463100050242);
}

__global__ void __launch_bounds__(256) load_family_kernel(int family, int N, int p,
                                                          const double* __restrict__ eta,
                                                          const double* __restrict__ ux,
                                                          const double* __restrict__ uv,
                                                          double* __restrict__ X,
                                                          double* __restrict__ V,
                                                          cplx* __restrict__ C) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)N * p) return;
  const int l = (int)(t % N), i = (int)(t / N);
  const double alpha = eta[4 * i], k = eta[4 * i + 1];
  const double v0 = (family == 0) ? 0.0 : eta[4 * i + 2], sg = eta[4 * i + 3];
  const double vmax = 10.0;
  // position
  const double L = 2.0 * M_PI / k;
  const double target = ux[l] * L;
  double x = target;
  for (int it = 0; it < 100; ++it) {
    const double g = x + (alpha / k) * sin(k * x) - target;
    const double dg = 1.0 + alpha * cos(k * x);
    const double step = g / dg;
    x = fmin(fmax(x - step, 0.0), L);
    if (fabs(step) <= 1e-15 * L) break;
  }
  // velocity
  const double lo_m = mix_cdf(-vmax, v0, sg), hi_m = mix_cdf(vmax, v0, sg);
  const double tv = lo_m + uv[l] * (hi_m - lo_m);
  double v;
  if (v0 == 0.0) {
    v = fmin(fmax(sg * normcdfinv(tv), -vmax), vmax);
  } else {
    if (tv < 0.5)
      v = -v0 + sg * normcdfinv(fmin(fmax(2.0 * tv, 1e-300), 1.0));
    else
      v = v0 + sg * normcdfinv(fmin(fmax(2.0 * tv - 1.0, 1e-300), 1.0 - 1e-16));
    if (!isfinite(v)) v = 0.0;
    v = fmin(fmax(v, -vmax), vmax);
    double lo = -vmax, hi = vmax;
    for (int it = 0; it < 200; ++it) {
      const double f = mix_cdf(v, v0, sg) - tv;
      if (f < 0.0)
        lo = v;
      else
        hi = v;
      const double d = mix_pdf(v, v0, sg);
      double vn = v - f / d;
      if (!isfinite(vn) || vn <= lo || vn >= hi) vn = 0.5 * (lo + hi);
      const bool hit = fabs(f) <= 1e-16;
      if (hit) vn = v;
      const bool done = hit || fabs(vn - v) <= 1e-12 * (1.0 + fabs(vn)) || hi - lo <= 1e-14;
      v = vn;
      if (done) break;
    }
  }
  if (X) X[t] = x;
  if (V) V[t] = v;
  if (C) C[t] = mk(x, v);
}

void launch_load_family(hipStream_t s, int family, int N, int p, const double* eta,
                        const double* ux, const double* uv, double* X, double* V, cplx* C) {
  const size_t tot = (size_t)N * p;
  hipLaunchKernelGGL(load_family_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     family, N, p, eta, ux, uv, X, V, C);
}
