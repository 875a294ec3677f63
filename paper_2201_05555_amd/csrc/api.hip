// C ABI of the symrom library: workspace layout, handles and the host-side
// orchestration of the reduced step (Sec. 5) and of the full-order step
// (eq. sv_full_order).  All arithmetic of a step runs in the HIP kernels; the
// host only enqueues launches and reads the fixed-point counters.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/symrom.h"
#include "common.h"
#include "kernels.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static symrom_status fail(symrom_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(SYMROM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

#define LAUNCHCHK()                                                                     \
  do {                                                                                  \
    hipError_t _e = hipGetLastError();                                                  \
    if (_e != hipSuccess)                                                               \
      return fail(SYMROM_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(_e)); \
  } while (0)

extern "C" const char* symrom_status_string(symrom_status s) {
  switch (s) {
    case SYMROM_OK: return "ok";
    case SYMROM_EINVAL: return "invalid argument";
    case SYMROM_ENOMEM: return "workspace too small";
    case SYMROM_ESINGULAR: return "singular small matrix";
    case SYMROM_ENOCONV: return "fixed point not converged";
    case SYMROM_EDEVICE: return "device error";
    case SYMROM_ESTATE: return "bad handle state";
    case SYMROM_ERANKCAP: return "rank cap reached";
  }
  return "unknown status";
}

extern "C" const char* symrom_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// kernel timing (HIP events around launches of the instrumented families)
// ---------------------------------------------------------------------------
namespace {
struct TimedLaunch {
  int family;
  hipEvent_t a, b;
};
bool g_timing = false;
std::vector<TimedLaunch> g_pending;
std::vector<hipEvent_t> g_event_pool;
double g_ms[16] = {0};
int64_t g_launches[16] = {0};
double g_flops[16] = {0};
double g_bytes[16] = {0};

hipEvent_t take_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void drain_timing() {
  for (auto& t : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      g_ms[t.family] += ms;
      g_launches[t.family] += 1;
    }
    g_event_pool.push_back(t.a);
    g_event_pool.push_back(t.b);
  }
  g_pending.clear();
}

struct Timer {
  int fam;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  // flops / bytes: algorithmic work of the launches inside the scope
  Timer(int f, hipStream_t st, double flops = 0.0, double bytes = 0.0) : fam(f), s(st) {
    if (g_timing) {
      g_flops[f] += flops;
      g_bytes[f] += bytes;
      a = take_event();
      b = take_event();
      if (a) hipEventRecord(a, s);
    }
  }
  ~Timer() {
    if (g_timing && a && b) {
      hipEventRecord(b, s);
      g_pending.push_back({fam, a, b});
      if (g_pending.size() > 4096) drain_timing();
    }
  }
};
}  // namespace

enum {
  FAM_DEPOSIT = 0,
  FAM_GATHER = 1,
  FAM_POISSON = 2,
  FAM_FOMPUSH = 3,
  FAM_BASIS = 4,
  FAM_DENSE = 5,
  FAM_EIG = 6,
  FAM_XI = 7,
  FAM_CHAIN = 8,
  FAM_DMD = 9,     // DMD of the subset potentials and the predicted field tables
  FAM_DMDFP = 10,  // the fused fixed point with the DMD-DEIM gradient
  NFAM = 11
};

extern "C" void symrom_set_timing(int32_t on) {
  drain_timing();
  g_timing = on != 0;
}

extern "C" double symrom_kernel_ms(int32_t family, int64_t* launches) {
  drain_timing();
  if (family < 0 || family >= NFAM) return 0.0;
  double v = g_ms[family];
  if (launches) *launches = g_launches[family];
  g_ms[family] = 0.0;
  g_launches[family] = 0;
  return v;
}

extern "C" void symrom_kernel_work(int32_t family, double* flops, double* bytes) {
  if (family < 0 || family >= NFAM) return;
  if (flops) *flops = g_flops[family];
  if (bytes) *bytes = g_bytes[family];
  g_flops[family] = 0.0;
  g_bytes[family] = 0.0;
}

// ---------------------------------------------------------------------------
// workspace carving (a dry run with base == nullptr measures the size)
// ---------------------------------------------------------------------------
namespace {
struct Arena {
  char* base;
  size_t off = 0;
  explicit Arena(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

PicGeom pic_geom(int N, int p, int Nx, size_t lds_per_table_budget, int min_blocks) {
  PicGeom g;
  int pt = (int)(lds_per_table_budget / ((size_t)Nx * sizeof(double)));
  if (pt < 1) pt = 1;
  if (pt > p) pt = p;
  g.pt = pt;
  int ntiles = (p + pt - 1) / pt;
  // row blocks: enough blocks to fill 256 CUs twice, at least 256 rows each
  int nrb = (min_blocks + ntiles - 1) / ntiles;
  int max_nrb = (N + 255) / 256;
  if (nrb > max_nrb) nrb = max_nrb;
  if (nrb < 1) nrb = 1;
  // fewer than 2^24 rows per block (the deterministic deposit's integer
  // theta sums stay below 2^64)
  const int min_nrb = (int)((N + (1 << 24) - 2) / ((1 << 24) - 1));
  if (nrb < min_nrb) nrb = min_nrb;
  g.rpb = (N + nrb - 1) / nrb;
  g.nrb = (N + g.rpb - 1) / g.rpb;
  return g;
}

void per_param_consts(const double* L, int N, int p, int Nx, double q, double m,
                      std::vector<double>& factor, std::vector<double>& qw, std::vector<double>& h,
                      std::vector<double>& mw) {
  factor.resize(p);
  qw.resize(p);
  h.resize(p);
  mw.resize(p);
  for (int i = 0; i < p; ++i) {
    factor[i] = (double)Nx / L[i];
    const double w = L[i] / (double)N;
    qw[i] = q * w;
    h[i] = L[i] / (double)Nx;
    mw[i] = m * w;
  }
}
}  // namespace

// ---------------------------------------------------------------------------
// stateless particle-to-grid
// ---------------------------------------------------------------------------
namespace {
struct PicBufs {
  double *factor, *qw, *h, *mw, *part, *rho, *phi, *e, *energy;
};
PicBufs carve_pic(Arena& ar, int N, int p, int Nx, const PicGeom& g) {
  PicBufs b;
  b.factor = ar.take<double>(p);
  b.qw = ar.take<double>(p);
  b.h = ar.take<double>(p);
  b.mw = ar.take<double>(p);
  // deposit partials + their row-block sums; also scratch for column sums
  size_t np_ = (size_t)(g.nrb + 1) * p * Nx;
  if (np_ < (size_t)32 * p) np_ = (size_t)32 * p;
  b.part = ar.take<double>(np_);
  b.rho = ar.take<double>((size_t)p * Nx);
  b.phi = ar.take<double>((size_t)p * Nx);
  b.e = ar.take<double>((size_t)p * Nx);
  b.energy = ar.take<double>(p);
  return b;
}
const size_t kFomTableBudget = 16 * 1024;  // LDS bytes per table (field and histogram)
const size_t kDepTableBudget = 64 * 1024;
bool valid_sizes(int N, int p, int Nx) {
  return N > 0 && p > 0 && Nx >= 2 && Nx <= SYMROM_MAX_NX;
}
}  // namespace

extern "C" size_t pic_workspace_bytes(int32_t N, int32_t p, int32_t Nx) {
  if (!valid_sizes(N, p, Nx)) return 0;
  Arena ar(nullptr);
  PicGeom g = pic_geom(N, p, Nx, kDepTableBudget, 512);
  carve_pic(ar, N, p, Nx, g);
  return ar.off + 256;
}

extern "C" symrom_status pic_fields(int32_t N, int32_t p, int32_t Nx, const double* L, double q,
                                    const double* X, int32_t* cells, double* rho, double* Phi,
                                    double* e, void* ws, size_t ws_bytes, void* stream) {
  if (!valid_sizes(N, p, Nx) || !L || !X) return fail(SYMROM_EINVAL, "pic_fields: bad arguments");
  size_t need = pic_workspace_bytes(N, p, Nx);
  if (!ws || ws_bytes < need) return fail(SYMROM_ENOMEM, "pic_fields: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  Arena ar(ws);
  PicGeom g = pic_geom(N, p, Nx, kDepTableBudget, 512);
  PicBufs b = carve_pic(ar, N, p, Nx, g);
  std::vector<double> factor, qw, h, mw;
  per_param_consts(L, N, p, Nx, q, 1.0, factor, qw, h, mw);
  HIPCHK(hipMemcpyAsync(b.factor, factor.data(), p * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(b.qw, qw.data(), p * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(b.h, h.data(), p * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(b.mw, mw.data(), p * sizeof(double), hipMemcpyHostToDevice, s));
  {
    Timer t(FAM_DEPOSIT, s);
    launch_deposit_x(s, X, N, p, Nx, g, b.factor, b.part);
  }
  {
    Timer t(FAM_POISSON, s);
    launch_poisson(s, b.part, g.nrb, p, Nx, b.qw, b.h, b.mw, nullptr, rho ? rho : b.rho,
                   Phi ? Phi : b.phi, e ? e : b.e, b.energy);
  }
  if (cells) launch_cells(s, X, N, p, Nx, b.factor, cells);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  return SYMROM_OK;
}

// ---------------------------------------------------------------------------
// stateless particle-to-grid without allocation: the deposit partials, the
// per-parameter constants and the energies live in `scratch`, a file-scope
// device array of SYMROM_NOALLOC_SCRATCH_BYTES that each GPU holds until the
// process ends.  Its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// passed to kernels.  Calls that overlap on one GPU share the array and race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[SYMROM_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// device address of this device's scratch array (nullptr on failure)
symrom_status scratch_address(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SYMROM_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(SYMROM_EDEVICE, "scratch array has no device address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SYMROM_OK;
}

// per-parameter constants from the device array L (as per_param_consts)
__global__ void pic_consts_kernel(const double* __restrict__ L, int N, int p, int Nx, double q,
                                  double* __restrict__ factor, double* __restrict__ qw,
                                  double* __restrict__ h, double* __restrict__ mw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p) return;
  const double Li = L[i];
  factor[i] = (double)Nx / Li;
  const double w = Li / (double)N;
  qw[i] = q * w;
  h[i] = Li / (double)Nx;
  mw[i] = w;
}

// the row-block geometry of pic_fields, with fewer row blocks when the
// partials would not fit the scratch array; false when even one does not
bool noalloc_geom(int N, int p, int Nx, PicGeom& g) {
  g = pic_geom(N, p, Nx, kDepTableBudget, 512);
  const int ntiles = (p + g.pt - 1) / g.pt;
  (void)ntiles;
  for (;;) {
    Arena ar(nullptr);
    carve_pic(ar, N, p, Nx, g);
    if (ar.off + 256 <= SYMROM_NOALLOC_SCRATCH_BYTES) return true;
    if (g.nrb == 1) return false;
    const int nrb = std::max(1, g.nrb / 2);
    g.rpb = (N + nrb - 1) / nrb;
    g.nrb = (N + g.rpb - 1) / g.rpb;
  }
}
}  // namespace

extern "C" symrom_status pic_fields_noalloc(int32_t N, int32_t p, int32_t Nx, const double* L,
                                            double q, const double* X, int32_t* cells,
                                            double* rho, double* Phi, double* e, void* stream) {
  if (!valid_sizes(N, p, Nx) || !L || !X)
    return fail(SYMROM_EINVAL, "pic_fields_noalloc: bad arguments");
  PicGeom g;
  if (!noalloc_geom(N, p, Nx, g))
    return fail(SYMROM_EINVAL, "pic_fields_noalloc: p * Nx too large for the " +
                                   std::to_string(SYMROM_NOALLOC_SCRATCH_BYTES >> 20) +
                                   " MiB scratch array (use pic_fields with a workspace)");
  void* base = nullptr;
  symrom_status st = scratch_address(&base);
  if (st != SYMROM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar(base);
  PicBufs b = carve_pic(ar, N, p, Nx, g);
  // every scratch word read below is written first by this call
  hipLaunchKernelGGL(pic_consts_kernel, dim3((p + 255) / 256), dim3(256), 0, s, L, N, p, Nx, q,
                     b.factor, b.qw, b.h, b.mw);
  launch_deposit_x(s, X, N, p, Nx, g, b.factor, b.part);
  launch_poisson(s, b.part, g.nrb, p, Nx, b.qw, b.h, b.mw, nullptr, rho ? rho : b.rho,
                 Phi ? Phi : b.phi, e ? e : b.e, b.energy);
  if (cells) launch_cells(s, X, N, p, Nx, b.factor, cells);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  return SYMROM_OK;
}

// ---------------------------------------------------------------------------
// full-order model
// ---------------------------------------------------------------------------
struct symrom_fom {
  int N, p, Nx;
  double dt, q, m;
  hipStream_t s;
  PicGeom g;   // push geometry
  PicBufs b;
  double *X, *V;  // V holds the staggered velocity V_{t - dt/2}
  double* Vtmp;
  int64_t step;
};

namespace {
void carve_fom(Arena& ar, symrom_fom& f) {
  f.g = pic_geom(f.N, f.p, f.Nx, kFomTableBudget, 512);
  f.b = carve_pic(ar, f.N, f.p, f.Nx, f.g);
  f.X = ar.take<double>((size_t)f.N * f.p);
  f.V = ar.take<double>((size_t)f.N * f.p);
  f.Vtmp = ar.take<double>((size_t)f.N * f.p);
}
}  // namespace

extern "C" size_t fom_workspace_bytes(int32_t N, int32_t p, int32_t Nx) {
  if (!valid_sizes(N, p, Nx)) return 0;
  symrom_fom f{};
  f.N = N;
  f.p = p;
  f.Nx = Nx;
  Arena ar(nullptr);
  carve_fom(ar, f);
  return ar.off + 256;
}

namespace {
// fill(f): writes the initial X, V into f.X, f.V on f.s
symrom_status fom_init_impl(int32_t N, int32_t p, int32_t Nx, double dt, double q, double m,
                            const double* L, const std::function<bool(symrom_fom&)>& fill,
                            void* ws, size_t ws_bytes, void* stream, symrom_fom** out) {
  if (!valid_sizes(N, p, Nx) || !L || !out || !(m != 0.0))
    return fail(SYMROM_EINVAL, "fom_init: bad arguments");
  for (int i = 0; i < p; ++i)
    if (!(L[i] > 0.0) || !std::isfinite(L[i])) return fail(SYMROM_EINVAL, "fom_init: bad L");
  if (!ws || ws_bytes < fom_workspace_bytes(N, p, Nx))
    return fail(SYMROM_ENOMEM, "fom_init: workspace too small");
  symrom_fom* f = new symrom_fom{};
  f->N = N;
  f->p = p;
  f->Nx = Nx;
  f->dt = dt;
  f->q = q;
  f->m = m;
  f->s = (hipStream_t)stream;
  f->step = 0;
  Arena ar(ws);
  carve_fom(ar, *f);
  std::vector<double> factor, qw, h, mw;
  per_param_consts(L, N, p, Nx, q, m, factor, qw, h, mw);
  hipStream_t s = f->s;
  auto cleanup = [&](symrom_status st) {
    delete f;
    return st;
  };
  if (hipMemcpyAsync(f->b.factor, factor.data(), p * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(f->b.qw, qw.data(), p * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(f->b.h, h.data(), p * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(f->b.mw, mw.data(), p * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      !fill(*f))
    return cleanup(fail(SYMROM_EDEVICE, "fom_init: copy failed"));
  PicGeom gd = f->g;
  launch_deposit_x(s, f->X, N, p, Nx, gd, f->b.factor, f->b.part);
  launch_poisson(s, f->b.part, gd.nrb, p, Nx, f->b.qw, f->b.h, f->b.mw, nullptr, f->b.rho,
                 f->b.phi, f->b.e, f->b.energy);
  // staggered velocity V_{-1/2} = V_0 - dt/2 a(X_0)
  launch_fom_push(s, f->X, f->V, N, p, Nx, f->g, f->b.factor, f->b.e, q / m, -0.5 * dt, 0.0,
                  nullptr);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return cleanup(fail(SYMROM_EDEVICE, "fom_init: launch"));
  *out = f;
  return SYMROM_OK;
}

}  // namespace

extern "C" symrom_status fom_init(int32_t N, int32_t p, int32_t Nx, double dt, double q, double m,
                                  const double* L, const double* X0, const double* V0, void* ws,
                                  size_t ws_bytes, void* stream, symrom_fom** out) {
  if (!X0 || !V0) return fail(SYMROM_EINVAL, "fom_init: null state");
  auto fill = [&](symrom_fom& f) {
    return hipMemcpyAsync(f.X, X0, (size_t)N * p * 8, hipMemcpyDeviceToDevice, f.s) ==
               hipSuccess &&
           hipMemcpyAsync(f.V, V0, (size_t)N * p * 8, hipMemcpyDeviceToDevice, f.s) == hipSuccess;
  };
  return fom_init_impl(N, p, Nx, dt, q, m, L, fill, ws, ws_bytes, stream, out);
}

// L_i = 2 pi / k_i from eta (host, p x 4: alpha, k, v0, sigma); false when
// a wave number or a spread is not positive or a value is not finite
namespace {
bool eta_lengths(int p, const double* eta, std::vector<double>& L) {
  L.resize(p);
  for (int i = 0; i < p; ++i) {
    for (int c = 0; c < 4; ++c)
      if (!std::isfinite(eta[4 * i + c])) return false;
    if (!(eta[4 * i + 1] > 0.0) || !(eta[4 * i + 3] > 0.0)) return false;
    L[i] = 2.0 * M_PI / eta[4 * i + 1];
  }
  return true;
}
}  // namespace

extern "C" symrom_status fom_init_family(int32_t N, int32_t p, int32_t Nx, double dt, double q,
                                         double m, int32_t family, const double* eta,
                                         const double* ux, const double* uv, void* ws,
                                         size_t ws_bytes, void* stream, symrom_fom** out) {
  std::vector<double> L;
  if (!eta || !ux || !uv || (family != 0 && family != 1) || !valid_sizes(N, p, Nx) ||
      !eta_lengths(p, eta, L))
    return fail(SYMROM_EINVAL, "fom_init_family: bad arguments");
  // eta is staged in the deposit-partials buffer (at least 32 p doubles),
  // which the first deposit overwrites only after the load has read it
  auto fill = [&](symrom_fom& f) {
    if (hipMemcpyAsync(f.b.part, eta, (size_t)4 * p * sizeof(double), hipMemcpyHostToDevice,
                       f.s) != hipSuccess)
      return false;
    launch_load_family(f.s, family, N, p, f.b.part, ux, uv, f.X, f.V, nullptr);
    return hipGetLastError() == hipSuccess;
  };
  return fom_init_impl(N, p, Nx, dt, q, m, L.data(), fill, ws, ws_bytes, stream, out);
}

extern "C" symrom_status fom_step(symrom_fom* f, int32_t nsteps) {
  if (!f || nsteps < 0) return fail(SYMROM_EINVAL, "fom_step: bad arguments");
  hipStream_t s = f->s;
  for (int it = 0; it < nsteps; ++it) {
    {
      const double pp = (double)f->N * f->p;
      Timer t(FAM_FOMPUSH, s, 12.0 * pp,
              32.0 * pp + 8.0 * (double)f->g.nrb * f->p * f->Nx);
      launch_fom_push(s, f->X, f->V, f->N, f->p, f->Nx, f->g, f->b.factor, f->b.e, f->q / f->m,
                      f->dt, f->dt, f->b.part);
    }
    {
      Timer t(FAM_POISSON, s);
      launch_poisson(s, f->b.part, f->g.nrb, f->p, f->Nx, f->b.qw, f->b.h, f->b.mw, nullptr,
                     f->b.rho, f->b.phi, f->b.e, f->b.energy);
    }
    f->step++;
  }
  LAUNCHCHK();
  return SYMROM_OK;
}

extern "C" symrom_status fom_get_state(symrom_fom* f, double* X, double* V) {
  if (!f) return fail(SYMROM_EINVAL, "fom_get_state: null handle");
  hipStream_t s = f->s;
  size_t n = (size_t)f->N * f->p;
  if (X) HIPCHK(hipMemcpyAsync(X, f->X, n * 8, hipMemcpyDeviceToDevice, s));
  if (V)
    launch_fom_velocity(s, f->X, f->V, f->N, f->p, f->Nx, f->b.factor, f->b.e, f->q / f->m,
                        0.5 * f->dt, V);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  return SYMROM_OK;
}

extern "C" symrom_status fom_diagnostics(symrom_fom* f, double* E, double* H) {
  if (!f) return fail(SYMROM_EINVAL, "fom_diagnostics: null handle");
  hipStream_t s = f->s;
  if (E) HIPCHK(hipMemcpyAsync(E, f->b.energy, f->p * 8, hipMemcpyDeviceToDevice, s));
  if (H) {
    launch_fom_velocity(s, f->X, f->V, f->N, f->p, f->Nx, f->b.factor, f->b.e, f->q / f->m,
                        0.5 * f->dt, f->Vtmp);
    launch_colsumsq(s, f->Vtmp, f->N, f->p, 0.5, H, f->b.part);
    launch_vec_add(s, H, f->b.energy, f->p);
  }
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  return SYMROM_OK;
}

extern "C" void fom_destroy(symrom_fom* f) { delete f; }

// ---------------------------------------------------------------------------
// reduced model
// ---------------------------------------------------------------------------
struct symrom_rom {
  symrom_config cfg;
  int N, p, Nx, n, nmax;
  hipStream_t s;
  int64_t step;
  bool ready;
  PicGeom gdep, ggat;
  int nkb;
  PicBufs b;
  // N x nmax complex
  cplx *U0, *Uh, *Xi, *P, *Xv, *Ups;
  cplx* G;  // N x p complex
  // nmax x p complex
  cplx *Z0, *Zev, *ZG, *k, *Z1, *gproj;
  cplx* Q;  // p x nmax
  double* prev;
  int* active;
  // status block (device, 16 ints; [0..11] read back in one copy): flags
  // [0] error bits, [1] eigen path, [2] error bits of the DEIM chain of the
  // step, [3] those of the DEIM chain in flight (folded into [2] at the end of
  // its step, so that a chain enqueued ahead never mixes with the step
  // before it); counters [0] active
  // left, [1] stalled, [2] iterations run; eps_dev the rank indicator;
  // [12] the stop word of a head enqueued ahead (nonzero: the step failed)
  int* status;
  int* counters;
  int* flags;
  int* hstat;  // pinned host mirror of the status block
  cplx *Gram, *Amat, *MU, *MX, *M1, *M2, *M3, *C0x, *MP;
  cplx* gemm_part;
  double* sigma2;
  double* eps_dev;
  // init scratch
  cplx *Gp, *Vp;
  double* lam;
  int n_active;  // active fixed-point columns (host copy, for work accounting)
  int fp_hint;   // iterations the last fixed point took (speculative batch size)
  bool stage1_cached;  // G, g and the fields in the buffers belong to (U0, Z0)
  double* colsq;       // per-parameter |G~|^2
  // DEIM (Sec. 4.2.2): snapshot ring of T+1 slots (N x psub each) and operator
  int psub, nslots, win_count, d_cur;
  bool deim_on;
  int* sub;
  double* Ywin;
  double* Psi;
  int* didx;
  double *dw, *dc, *bval, *colpart, *Mdeim, *ylam;
  double *dB, *dcv;  // ping-pong (P^T Psi)^{-1} (64 x 64) and coefficient vectors of the greedy passes
  int* bidx;
  int nbg, nbc;
  cplx *YG, *YV, *C12, *C12a, *gF;
  cplx* C12t;  // the Grams of a basis passed to full_gradient without its own
  double* dpart;  // split-K partials of the DEIM Gram (its own: the chain runs beside the main work)
  // The DEIM operator is built on a second stream (default priority) beside
  // the basis velocity and Cayley map of the same step, which do not need it;
  // ev_fork / ev_join order it after the first-stage field and before its use.
  hipStream_t s2;
  hipEvent_t ev_fork, ev_join;
  // DMD-DEIM: the DMD of the potential window on a third stream (default
  // priority) beside the DEIM chain; both need only the first-stage field
  hipStream_t s3;
  hipEvent_t ev_join3;
  // S(Z)^+ of the second-stage basis velocity on the second stream, beside
  // the gather-projection that precedes it: ev_sp0 orders it after the fixed
  // point, ev_sp1 its result before the basis-velocity finish
  hipEvent_t ev_sp0, ev_sp1;
  hipEvent_t ev_read;  // end-of-step status copy done
  // With rank adaptation the first-stage field of the next step is known at
  // the end of a step: the head of the next DEIM update (snapshot, Gram
  // block, eigenpairs, coefficients) is then enqueued on the second stream
  // before the end-of-step readback, gated on the device by the stop word.
  // head_n: the rank it was built for (a rank change before the next step
  // means it is built again for the same slot).
  bool head_pending;
  int head_n;
  double* zsig;  // singular values of Z~ (automatic shrink)
  // adaptive DEIM (Sec. 4.2.2): double-buffered basis and indices, the d of
  // the operator in each buffer, the inherited indices, rotation partials
  double* Psib[2];
  int* didxb[2];
  int dbuf[2];
  int* forced;
  double* rotpart;
  // DMD-DEIM (Alg. 2).  The subset S of eq. pSampl sits in `sub` (psub = p*
  // entries, chosen at initialisation); sub_id is the identity of the
  // compact subset.  bs, gdep_s, ggat_s: the per-parameter buffers and
  // launch shapes of the p* compact columns Zs, used for the exact gradient
  // of the basis evolution.  phiw: the window levels of the subset
  // potentials (nslots blocks of p* x Nx, in the slots of the snapshot ring).
  int* sub_id;
  PicBufs bs;
  PicGeom gdep_s, ggat_s;
  cplx* Zs;
  double* phiw;
  DmdChainArgs dmd;
  double *e0, *eh;     // predicted field tables (p x Nx)
  double* beta;        // radial basis weights (p x p*)
  int* member;
  double* dmin;
  double* eta;         // parameters (p x eta_dim)
  int eta_dim;
  bool beta_ready;
  cplx* Ysub;    // Rayleigh-Ritz eigenvectors of the subspace iteration (64 x 64)
  cplx* Wsub;    // its p x 64 block of vectors (p > 64)
  double* lamsub;
  symrom_step_info last;
  std::vector<double> init_sig;  // singular values of C0 found by the initialisation
  // set during rom_step_hamiltonian_split: U_{tau-1/2} and Z_tau (before the
  // re-orthonormalisation) are copied here (caller's scratch)
  cplx* split_U = nullptr;
  cplx* split_Z = nullptr;
};

namespace {
// Size p* of the DEIM snapshot parameter subset: evenly spaced indices
// i_k = floor(k p / p*), p* = min(p, max(8, ceil(two_n_max / (T+1)))) so that
// the snapshot matrix (N x p*(T+1)) has at least d = 2n <= two_n_max columns.
int deim_psub(const symrom_config& c) {
  // DMD-DEIM: the subset of eq. pSampl, p* columns (all of them when 0)
  if (c.projection == SYMROM_DMD_DEIM) return (c.p_star > 0 && c.p_star < c.p) ? c.p_star : c.p;
  const int T1 = c.deim_window + 1;
  int ps = (c.two_n_max + T1 - 1) / T1;
  if (ps < 8) ps = 8;
  if (ps > c.p) ps = c.p;
  return ps;
}

int nkb_for(int N) {
  // split-K blocks: about one per CU, at least 64 rows each
  int nkb = (N + 63) / 64;
  if (nkb > 256) nkb = 256;
  if (nkb < 1) nkb = 1;
  return nkb;
}

void carve_rom(Arena& ar, symrom_rom& r) {
  const int N = r.N, p = r.p, Nx = r.Nx, nm = r.nmax;
  // one parameter tile of up to 64 KB of LDS per table, ~one block per CU
  // (row blocks for deposit tiles of deposit_tile_params(Nx) parameters)
  r.gdep = pic_geom(N, p, Nx, (size_t)deposit_tile_params(Nx) * Nx * sizeof(double), 256);
  r.ggat = pic_geom(N, p, Nx, 64 * 1024, 256);
  r.nkb = nkb_for(N);
  r.b = carve_pic(ar, N, p, Nx, r.gdep.nrb >= r.ggat.nrb ? r.gdep : r.ggat);
  const size_t Nn = (size_t)N * nm;
  r.U0 = ar.take<cplx>(Nn);
  r.Uh = ar.take<cplx>(Nn);
  r.Xi = ar.take<cplx>(Nn);
  r.P = ar.take<cplx>(Nn);
  r.Xv = ar.take<cplx>(Nn);
  r.Ups = ar.take<cplx>(Nn);
  r.G = ar.take<cplx>((size_t)N * p);
  const size_t np_ = (size_t)nm * p;
  r.Z0 = ar.take<cplx>(np_);
  r.Zev = ar.take<cplx>(np_);
  r.ZG = ar.take<cplx>(np_);
  r.k = ar.take<cplx>(np_);
  r.Z1 = ar.take<cplx>(np_);
  r.gproj = ar.take<cplx>(np_ > (size_t)p * p ? np_ : (size_t)p * p);
  r.Q = ar.take<cplx>((size_t)p * nm);
  r.prev = ar.take<double>(p);
  r.active = ar.take<int>(p);
  r.status = ar.take<int>(16);
  r.flags = r.status;
  r.counters = r.status + 4;
  r.eps_dev = reinterpret_cast<double*>(r.status + 8);
  // the largest Gram: [U0, xi, U_half, X]^* of the same (4n x 4n)
  const size_t m2 = (size_t)16 * nm * nm;
  r.Gram = ar.take<cplx>(m2 > (size_t)p * p ? m2 : (size_t)p * p);
  r.Amat = ar.take<cplx>((size_t)nm * nm);
  r.MU = ar.take<cplx>((size_t)nm * nm);
  r.MX = ar.take<cplx>((size_t)nm * nm);
  r.M1 = ar.take<cplx>((size_t)nm * nm);
  r.M2 = ar.take<cplx>((size_t)nm * nm);
  r.M3 = ar.take<cplx>((size_t)nm * nm);
  r.C0x = ar.take<cplx>((size_t)nm * nm);
  r.MP = ar.take<cplx>((size_t)nm * nm);
  // split-K partials: nkb * max(a*b) with a, b <= 64 (b chunked by 64)
  r.gemm_part = ar.take<cplx>((size_t)r.nkb * 64 * 64);
  r.sigma2 = ar.take<double>(nm);
  r.colsq = ar.take<double>(p);
  r.Gp = ar.take<cplx>((size_t)p * p);
  r.Vp = ar.take<cplx>((size_t)p * p);
  r.lam = ar.take<double>(p);
  // DEIM
  r.nslots = r.cfg.deim_window + 1;
  r.psub = deim_psub(r.cfg);
  const int P = r.psub * r.nslots;
  const int dmax = std::max(2 * nm, r.cfg.deim_rows);
  r.nbg = 256;
  r.nbc = 64;
  r.sub = ar.take<int>(r.psub);
  const bool dei = r.cfg.projection != SYMROM_GALERKIN;
  r.Ywin = ar.take<double>(dei ? (size_t)P * N : 0);
  // the DEIM basis and indices of two consecutive operators (the adaptive
  // update reads the previous ones): operator b uses buffer b % 2
  for (int q = 0; q < 2; ++q) {
    r.Psib[q] = ar.take<double>(dei ? (size_t)dmax * N : 0);
    r.didxb[q] = ar.take<int>(dmax);
  }
  r.Psi = r.Psib[0];
  r.didx = r.didxb[0];
  r.forced = ar.take<int>(dmax);
  r.rotpart = ar.take<double>((size_t)psi_blocks(r.N) * dmax);
  r.dw = ar.take<double>(dmax);
  r.dc = ar.take<double>(dmax);
  r.bval = ar.take<double>(2 * (size_t)r.nbg);
  r.dB = ar.take<double>(dei ? 2 * 64 * 64 : 0);
  r.dcv = ar.take<double>(dei ? 2 * 64 : 0);
  r.bidx = ar.take<int>(2 * (size_t)r.nbg);
  r.colpart = ar.take<double>((size_t)psi_blocks(r.N) * dmax);
  r.Mdeim = ar.take<double>((size_t)P * dmax);
  r.ylam = ar.take<double>(P);
  r.YG = ar.take<cplx>((size_t)P * P);
  r.YV = ar.take<cplx>((size_t)P * P);
  r.C12 = ar.take<cplx>((size_t)2 * nm * nm);
  r.C12a = ar.take<cplx>((size_t)2 * nm * nm);
  r.C12t = ar.take<cplx>((size_t)2 * nm * nm);
  r.gF = ar.take<cplx>((size_t)nm * p);
  r.zsig = ar.take<double>(nm);
  r.Ysub = ar.take<cplx>(64 * 64);
  r.Wsub = ar.take<cplx>(p > 64 ? (size_t)p * 64 : 0);
  r.lamsub = ar.take<double>(64);
  r.dpart = ar.take<double>(dei ? (size_t)r.nkb * 64 * 64 * 2 : 0);
  // DMD-DEIM
  const bool dm = r.cfg.projection == SYMROM_DMD_DEIM;
  const int ps = r.psub, T = r.cfg.deim_window, Pd = ps * T;
  r.sub_id = ar.take<int>(ps);
  r.gdep_s = pic_geom(N, ps, Nx, (size_t)deposit_tile_params(Nx) * Nx * sizeof(double), 256);
  r.ggat_s = pic_geom(N, ps, Nx, 64 * 1024, 256);
  r.bs = carve_pic(ar, dm ? N : 1, dm ? ps : 1, Nx,
                   r.gdep_s.nrb >= r.ggat_s.nrb ? r.gdep_s : r.ggat_s);
  r.Zs = ar.take<cplx>(dm ? (size_t)nm * ps : 0);
  r.phiw = ar.take<double>(dm ? (size_t)r.nslots * ps * Nx : 0);
  DmdChainArgs& c = r.dmd;
  c = DmdChainArgs{};
  const size_t nxp = dm ? (size_t)Nx * Pd : 0, pp = dm ? (size_t)Pd * Pd : 0;
  c.Y = ar.take<double>(nxp);
  c.Yp = ar.take<double>(nxp);
  c.W = ar.take<double>(nxp);
  c.sig = ar.take<double>(dm ? Pd : 0);
  c.V = ar.take<double>(pp);
  c.rdev = ar.take<int>(dm ? 4 : 0);
  c.B = ar.take<double>(nxp);
  c.U = ar.take<double>(nxp);
  c.A = ar.take<double>(pp);
  c.M = ar.take<double>(pp);
  c.lam = ar.take<cplx>(dm ? Pd : 0);
  c.Wb = ar.take<double>(nxp);
  c.Wf = ar.take<double>(dm ? (size_t)Nx * ps : 0);
  c.C = ar.take<double>(dm ? (size_t)Pd * ps : 0);
  c.BM = ar.take<double>(nxp);
  r.e0 = ar.take<double>(dm ? (size_t)p * Nx : 0);
  r.eh = ar.take<double>(dm ? (size_t)p * Nx : 0);
  r.beta = ar.take<double>(dm ? (size_t)p * ps : 0);
  r.member = ar.take<int>(dm ? p : 0);
  r.dmin = ar.take<double>(dm ? p : 0);
  r.eta = ar.take<double>(dm ? (size_t)8 * p : 0);
}

bool valid_rom_config(const symrom_config* c, std::string& why) {
  if (!c) {
    why = "null config";
    return false;
  }
  if (!valid_sizes(c->N, c->p, c->Nx)) {
    why = "sizes";
    return false;
  }
  if (c->two_n <= 0 || (c->two_n & 1) || c->two_n_max < c->two_n || (c->two_n_max & 1)) {
    why = "rank must be positive and even, two_n <= two_n_max";
    return false;
  }
  if (c->two_n_max > 60) {
    why = "two_n_max above 60 is not supported";
    return false;
  }
  if (c->two_n_max > 2 * c->N) {
    why = "rank above 2N";
    return false;
  }
  if (!(c->dt > 0.0) || !(c->m != 0.0) || !std::isfinite(c->dt)) {
    why = "dt, m";
    return false;
  }
  if (c->fp_max_iters < 1 || c->fp_fixed_iters < 0) {
    why = "fixed-point limits";
    return false;
  }
  if (c->projection != SYMROM_GALERKIN && c->projection != SYMROM_DEIM &&
      c->projection != SYMROM_DMD_DEIM) {
    why = "projection";
    return false;
  }
  if (!(c->fp_stall_tol >= 0.0) || !(c->rank_tol_down >= 0.0) || !(c->rank_tol_down < 1.0)) {
    why = "fp_stall_tol >= 0 and 0 <= rank_tol_down < 1";
    return false;
  }
  if (c->deim_rows < 0 || c->deim_rows > 64) {
    why = "deim_rows must be in 0..64 (0: d = 2n)";
    return false;
  }
  if (c->precision != SYMROM_FP64) {
    why = "precision: only SYMROM_FP64 arithmetic is built";
    return false;
  }
  if (c->deim_update_every < 0 || c->deim_update_rows < 0) {
    why = "deim_update_every and deim_update_rows must be >= 0";
    return false;
  }
  if (c->deterministic != 0 && c->deterministic != 1) {
    why = "deterministic must be 0 or 1";
    return false;
  }
  if (c->p > 4096) {
    why = "p above 4096 is not supported";
    return false;
  }
  if (c->projection == SYMROM_DMD_DEIM) {
    const int ps = deim_psub(*c), T = c->deim_window;
    if (T < 1 || T > 7) {
      why = "DMD-DEIM needs deim_window (T) in 1..7";
      return false;
    }
    if (c->p_star < 0 || ps * (T + 1) > 64 || ps * T > 48) {
      why = "DMD-DEIM needs p* (T+1) <= 64 and p* T <= 48";
      return false;
    }
    if (c->rank_auto) {
      why = "automatic rank adaptation is not built for DMD-DEIM";
      return false;
    }
    if (!(c->dmd_tol >= 0.0) || !(c->dmd_tol < 1.0)) {
      why = "dmd_tol must be in [0, 1)";
      return false;
    }
    if (c->two_n_max > 60) {
      why = "two_n_max above 60";
      return false;
    }
  }
  if (c->projection == SYMROM_DEIM) {
    if (c->deim_window < 0 || c->deim_window > 7) {
      why = "deim_window must be in 0..7";
      return false;
    }
    if (deim_psub(*c) * (c->deim_window + 1) > 64) {
      why = "DEIM snapshot matrix wider than 64 columns";
      return false;
    }
  }
  return true;
}

MatList ml(const cplx* a, int ca, const cplx* b = nullptr, int cb = 0) {
  MatList L{};
  L.ptr[0] = a;
  L.cols[0] = ca;
  L.count = 1;
  if (b) {
    L.ptr[1] = b;
    L.cols[1] = cb;
    L.count = 2;
  }
  return L;
}
MatList ml(const cplx* a, int ca, const cplx* b, int cb, const cplx* c, int cc, const cplx* d,
           int cd) {
  MatList L{};
  const cplx* pt[4] = {a, b, c, d};
  const int cl[4] = {ca, cb, cc, cd};
  for (int q = 0; q < 4; ++q) {
    L.ptr[q] = pt[q];
    L.cols[q] = cl[q];
  }
  L.count = 4;
  return L;
}

RowTerms rt(const cplx* in0, const cplx* M0, int k0, const cplx* in1 = nullptr,
            const cplx* M1 = nullptr, int k1 = 0, const cplx* in2 = nullptr,
            const cplx* M2 = nullptr, int k2 = 0) {
  RowTerms T{};
  T.in[0] = in0;
  T.M[0] = M0;
  T.k[0] = k0;
  T.count = 1;
  if (in1) {
    T.in[1] = in1;
    T.M[1] = M1;
    T.k[1] = k1;
    T.count = 2;
  }
  if (in2) {
    T.in[2] = in2;
    T.M[2] = M2;
    T.k[2] = k2;
    T.count = 3;
  }
  return T;
}

// The field of every column at (U, Z): deposit, then Poisson.
void full_gradient_field(symrom_rom& r, const cplx* U, const cplx* Z, const int* active,
                         const int* gate = nullptr, int* fold = nullptr) {
  hipStream_t s = r.s;
  const int n = r.n;
  {
    {
      // algorithmic work: 4n flops per (particle, parameter) for x; bytes:
      // U~ and Z~ read once, the charge of the active parameters written
      // (the per-row-block partial histograms are this design's traffic,
      // not the operation's)
      const double pact = (active ? (double)r.n_active : (double)r.p);
      Timer t(FAM_DEPOSIT, s, 4.0 * n * (double)r.N * pact,
              16.0 * n * ((double)r.N + r.p) + 8.0 * pact * r.Nx);
      launch_deposit_rom(s, U, r.N, n, Z, r.p, r.Nx, r.gdep, r.b.factor, active, r.b.part,
                         gate, fold, r.cfg.deterministic);
    }
    Timer t(FAM_POISSON, s);
    launch_poisson(s, r.b.part, r.gdep.nrb, r.p, r.Nx, r.b.qw, r.b.h, r.b.mw, active, r.b.rho,
                   r.b.phi, r.b.e, r.b.energy, gate);
  }
}

void linear_grams(symrom_rom& r, const cplx* U, cplx* C12);

// g = U^* G~ with the full gradient of every column at (U, Z): the field
// first when do_deposit (else the one in the buffers), then either the
// fused gather-projection (G~ never stored; the velocity part from the
// Grams G12 = [U^* U, U^T U] of this U, formed here into r.C12t when not
// given) or, for ranks beyond the fused kernels, the gather into r.G and a
// split-K product.  With want_colsq, |G~[:, c]|^2 goes to r.colsq.
void full_gradient(symrom_rom& r, const cplx* U, const cplx* Z, const int* active,
                   bool do_deposit, bool want_colsq = false, const int* gate = nullptr,
                   const cplx* G12 = nullptr) {
  hipStream_t s = r.s;
  const int n = r.n;
  const double qm = r.cfg.q / r.cfg.m;
  if (do_deposit) full_gradient_field(r, U, Z, active, gate);
  const double pact = (active ? (double)r.n_active : (double)r.p);
  if (fused_gradient_ok(n)) {
    if (!G12) {
      linear_grams(r, U, r.C12t);
      G12 = r.C12t;
    }
    // per (particle, parameter): 4n flops for x, 4n for the projection of
    // F, 2 for |F|^2; bytes: the basis and the coefficients read once, g
    // written (the field table, O(p Nx), is negligible)
    Timer t(FAM_GATHER, s, (8.0 * n + 2.0) * (double)r.N * pact,
            16.0 * n * ((double)r.N + 2.0 * r.p));
    launch_gather_project(s, U, r.N, n, Z, r.p, r.Nx, r.b.factor, r.b.e, qm, active, want_colsq,
                          r.gemm_part, (size_t)r.nkb * 64 * 64, r.gproj, r.colsq, G12, gate);
    return;
  }
  {
    const int ntiles = (r.p + r.ggat.pt - 1) / r.ggat.pt;
    Timer t(FAM_GATHER, s, 8.0 * n * (double)r.N * pact,
            16.0 * n * (double)r.N * ntiles + 16.0 * (double)r.N * pact);
    launch_gather_rom(s, U, r.N, n, Z, r.p, r.Nx, r.ggat, r.b.factor, r.b.e, qm, active, true,
                      r.G);
  }
  Timer t(FAM_BASIS, s);
  launch_gemm_ah_b(s, ml(U, n), n, ml(r.G, r.p), r.p, false, r.N, r.nkb, r.gemm_part, r.gproj);
  if (want_colsq)
    launch_colsumsq(s, reinterpret_cast<const double*>(r.G), 2 * r.N, r.p, 1.0, r.colsq, r.b.part);
}

// G~ at (U, Z) into r.G with the field already in r.b.e (for the rank
// growth, which needs G~^* G~ and G~ Q)
void materialise_gradient(symrom_rom& r, const cplx* U, const cplx* Z) {
  Timer t(FAM_BASIS, r.s);
  launch_gather_rom(r.s, U, r.N, r.n, Z, r.p, r.Nx, r.ggat, r.b.factor, r.b.e, r.cfg.q / r.cfg.m,
                    nullptr, true, r.G);
}

// X~ = -i (G~ Q - U T) scaled by `scale`, written to `out`, with G~ in r.G
// and g in r.gproj; Q = Z^* S(Z)^+ computed first.
// q_ready: S(Z)^+ Q has been formed already (and ordered before this call)
void basis_velocity(symrom_rom& r, const cplx* U, const cplx* Z, double scale, cplx* out,
                    cplx* k1, bool q_ready = false) {
  hipStream_t s = r.s;
  const int n = r.n;
  if (!q_ready) {
    Timer t(FAM_DENSE, s);
    launch_dense_spinv(s, Z, n, r.p, r.cfg.pinv_rtol, r.Q, r.sigma2, r.flags);
  }
  if (fused_gradient_ok(n)) {
    if (k1) {
      Timer t(FAM_DENSE, s);
      launch_dense_xfinish(s, r.gproj, r.Q, n, r.p, 2.0 * scale, k1, r.MP, r.MU);
    }
    // per (particle, parameter): 4n flops for x, 4n for F (-i h Q); plus
    // 16n^2 per particle for U M + conj(U) N; bytes: U read, out written.
    // Without k1 the kernel forms MU from g~ and Q itself (no separate launch).
    Timer t(FAM_XI, s, 8.0 * n * (double)r.N * r.p + 16.0 * n * n * (double)r.N,
            32.0 * n * (double)r.N);
    launch_gather_xi(s, U, r.N, n, Z, r.p, r.Nx, r.b.factor, r.b.e, r.cfg.q / r.cfg.m, r.Q, r.MU,
                     scale, out, k1 ? nullptr : r.gproj);
    return;
  }
  Timer t(FAM_BASIS, s);
  launch_rowgemm(s, rt(r.G, r.Q, r.p), r.N, n, r.P);  // P = G~ Q
  launch_dense_xfinish(s, r.gproj, r.Q, n, r.p, 2.0 * scale, k1, r.MP, r.MU);
  launch_rowgemm(s, rt(r.P, r.MP, n, U, r.MU, n), r.N, n, out);
}

// U_out = R_{U0}(xi) (Cayley retraction); A_out receives U0^* xi.
// gram_ready: r.Gram already holds [U0, xi]^* [U0, xi].
void cayley(symrom_rom& r, const cplx* U0, const cplx* xi, cplx* Uout, cplx* A_out,
            bool gram_ready = false) {
  hipStream_t s = r.s;
  const int n = r.n;
  Timer t(FAM_BASIS, s);
  if (!gram_ready)
    launch_gemm_ah_b(s, ml(U0, n, xi, n), 2 * n, ml(U0, n, xi, n), 2 * n, false, r.N, r.nkb,
                     r.gemm_part, r.Gram);
  launch_dense_cayley(s, r.Gram, n, A_out, r.MU, r.MX, r.flags);
  launch_rowgemm(s, rt(U0, r.MU, n, xi, r.MX, n), r.N, n, Uout);
}

// Uout = R_{U0}(xi) followed by two Cholesky-QR passes with Z <- R Z, the
// first without a pass over the rows: its Gram comes from the retraction's
// own Gram (U = U0 MU + xi MX gives U^* U = [MU; MX]^* [U0, xi]^* [U0, xi]
// [MU; MX]), and R^{-1} is folded into MU, MX, so that one row combination
// forms the once-factored basis.  Needs 4n <= 64 (the Gram of [U0, xi] and
// the row combination as for cayley).
void cayley_cholqr2(symrom_rom& r, const cplx* U0, const cplx* xi, cplx* Uout, cplx* A_out,
                    cplx* Z, bool gram_ready = false) {
  hipStream_t s = r.s;
  const int n = r.n;
  Timer t(FAM_BASIS, s);
  if (!gram_ready)
    launch_gemm_ah_b(s, ml(U0, n, xi, n), 2 * n, ml(U0, n, xi, n), 2 * n, false, r.N, r.nkb,
                     r.gemm_part, r.Gram);
  launch_dense_cayley(s, r.Gram, n, A_out, r.MU, r.MX, r.flags, true, Z, r.p);
  // the once-factored basis and, in the same pass, its Gram for the second
  if (!launch_rowgemm_gram(s, rt(U0, r.MU, n, xi, r.MX, n), r.N, n, Uout, r.gemm_part,
                           (size_t)r.nkb * 64 * 64, r.Gram)) {
    launch_rowgemm(s, rt(U0, r.MU, n, xi, r.MX, n), r.N, n, Uout);
    launch_gemm_ah_b(s, ml(Uout, n), n, ml(Uout, n), n, false, r.N, r.nkb, r.gemm_part, r.Gram);
  }
  launch_cholqr_apply(s, r.Gram, n, Uout, r.N, Z, r.p, r.flags);
}

// two Cholesky-QR passes on U (N x n) with Z <- R Z
void cholqr2(symrom_rom& r, cplx* U, cplx* Z) {
  hipStream_t s = r.s;
  const int n = r.n;
  Timer t(FAM_BASIS, s);
  for (int pass = 0; pass < 2; ++pass) {
    launch_gemm_ah_b(s, ml(U, n), n, ml(U, n), n, false, r.N, r.nkb, r.gemm_part, r.Gram);
    launch_cholqr_apply(s, r.Gram, n, U, r.N, Z, r.p, r.flags);
  }
}

// C12 = [U~^* U~, U~^T U~] (n x n each) for the linear part of the gradient
void linear_grams(symrom_rom& r, const cplx* U, cplx* C12) {
  hipStream_t s = r.s;
  const int n = r.n;
  Timer t(FAM_BASIS, s);
  launch_gemm_flags(s, ml(U, n), n, ml(U, n), n, 0, r.N, r.nkb, r.gemm_part, C12);
  launch_gemm_flags(s, ml(U, n), n, ml(U, n), n, GEMM_NO_CONJ_A, r.N, r.nkb, r.gemm_part,
                    C12 + (size_t)n * n);
}

// Snapshot at the start of a step into the ring, and when T+1 snapshots are
// held, the DEIM operator of this step: Psi = first d left singular vectors
// of Y (from the eigenpairs of Y^T Y), greedy indices, weights.  Enqueued on
// the second stream, with its own partials and its own error word flags[2].
void deim_update(symrom_rom& r, const cplx* U, const cplx* Z, bool redo = false,
                 const int* stop = nullptr, bool copy_phi = true) {
  hipStream_t s = r.s2;
  int* dflags = r.flags + 3;
  const int N = r.N, n = r.n;
  // redo: the snapshot of the newest slot again (the state changed after a
  // head built ahead of its step)
  const int slot = (redo ? r.win_count - 1 : r.win_count) % r.nslots;
  double* Ys = r.Ywin + (size_t)slot * r.psub * N;
  {
    Timer t(FAM_CHAIN, s);
    launch_snapshot(s, U, N, n, Z, r.sub, r.psub, r.Nx, r.b.factor, r.b.phi, Ys, stop);
    // DMD-DEIM: the subset potentials of this level into the same slot of
    // the potential window (eq. DMD_potential_Y_time)
    if (r.cfg.projection == SYMROM_DMD_DEIM && copy_phi)
      launch_grid_rows(s, r.b.phi, r.sub, r.psub, r.Nx, r.phiw + (size_t)slot * r.psub * r.Nx);
  }
  if (!redo) r.win_count++;
  const int P = r.psub * r.nslots;
  std::vector<const double*> slots(r.nslots);
  for (int q = 0; q < r.nslots; ++q) slots[q] = r.Ywin + (size_t)q * r.psub * N;
  {
    // the Gram Y^T Y (real, P x P) is kept across steps: only the row and
    // column block of the overwritten slot changes
    Timer t(FAM_CHAIN, s);
    launch_gram_block_real(s, Ys, slots.data(), r.nslots, r.psub, N, slot * r.psub,
                           r.nkb * 64 * 64 * 2, r.dpart, reinterpret_cast<double*>(r.YG), stop);
  }
  r.deim_on = r.win_count >= r.nslots;
  if (!r.deim_on) return;
  const int dreq = r.cfg.deim_rows > 0 ? r.cfg.deim_rows : 2 * n;
  const int d = (dreq < P) ? dreq : P;
  r.d_cur = d;
  {
    const double fP = P, fd = d;
    Timer te(FAM_EIG, s, 4.0 * fP * fP * fP / 3.0 + 2.0 * fP * fP * fd + 2.0 * fP * fd * fd,
             8.0 * fP * fP + 8.0 * fP * fd);
    // eigenpairs and the basis coefficients M = V diag(lambda)^{-1/2} in one launch
    launch_dense_topeig(s, reinterpret_cast<const double*>(r.YG), P, d,
                        reinterpret_cast<double*>(r.YV), r.ylam, dflags, stop, r.Mdeim);
  }
}

// Second half of the DEIM operator (after deim_update, same stream).
void deim_update_tail(symrom_rom& r) {
  if (!r.deim_on) return;
  hipStream_t s = r.s2;
  int* dflags = r.flags + 3;
  const int N = r.N, d = r.d_cur;
  std::vector<const double*> slots(r.nslots);
  for (int q = 0; q < r.nslots; ++q) slots[q] = r.Ywin + (size_t)q * r.psub * N;
  const int P = r.psub * r.nslots;
  Timer t(FAM_CHAIN, s);
  // operator b = win_count - nslots (0 for the first DEIM step; a rebuild of
  // the same step keeps b, a failed step takes it back) goes to buffer b % 2
  const int b = r.win_count - r.nslots;
  const int cur = b & 1, old = cur ^ 1;
  r.Psi = r.Psib[cur];
  r.didx = r.didxb[cur];
  const int kfull = std::max(1, r.cfg.deim_update_every);
  const bool full = kfull == 1 || b % kfull == 0 || r.dbuf[old] != d || r.cfg.deim_update_rows >= d;
  r.dbuf[cur] = d;
  // Psi and its column sums.  No sign convention is applied to the columns:
  // flipping the sign of column k negates c_k and the residual exactly, so
  // the greedy indices and the weights are the same bit for bit.
  launch_psi_colsum(s, slots.data(), r.nslots, r.psub, N, r.Mdeim, P, d, r.Psi, r.colpart);
  // between full selections only the positions of the most rotated basis
  // vectors are chosen again; the others inherit the previous indices
  const int* forced = nullptr;
  if (!full) {
    launch_deim_forced(s, r.Psi, r.Psib[old], N, d, std::max(0, r.cfg.deim_update_rows),
                       r.didxb[old], r.rotpart, r.forced, nullptr);
    forced = r.forced;
  }
  // greedy selection, one launch per index; block results ping-pong between
  // the two halves of bval / bidx
  // the inverse of P^T Psi and the coefficients ping-pong as well (pass k
  // reads those of pass k-1)
  for (int k = 0; k < d; ++k) {
    const int cur = k & 1, prev = cur ^ 1;
    launch_deim_greedy(s, r.Psi, N, k, r.didx, r.bval + prev * r.nbg, r.bidx + prev * r.nbg,
                       r.nbg, r.nbg, r.bval + cur * r.nbg, r.bidx + cur * r.nbg,
                       r.dB + prev * 4096, r.dcv + prev * 64, r.dB + cur * 4096,
                       r.dcv + cur * 64, dflags, forced);
  }
  const int last = (d - 1) & 1;
  launch_deim_weights(s, r.Psi, N, d, r.didx, r.bval + last * r.nbg, r.bidx + last * r.nbg,
                      r.nbg, r.dB + last * 4096, r.dcv + last * 64, r.colpart, psi_blocks(N),
                      r.dw, dflags, forced);
}

// the whole status block into the pinned mirror (one copy, one wait)
symrom_status read_status(symrom_rom& r) {
  HIPCHK(hipMemcpyAsync(r.hstat, r.status, 12 * sizeof(int), hipMemcpyDeviceToHost, r.s));
  HIPCHK(hipStreamSynchronize(r.s));
  return SYMROM_OK;
}

symrom_status read_flags(symrom_rom& r, int* host) {
  symrom_status st = read_status(r);
  host[0] = r.hstat[0] | r.hstat[2];
  host[1] = r.hstat[1];
  return st;
}

symrom_status rom_grow_apply(symrom_rom& r, int k);
symrom_status rom_shrink(symrom_rom& r, int n_new);
symrom_status shrink_exact(symrom_rom& r);

// Certificate of the automatic shrink for the current Z0 into status word 13
// (0: nothing can be dropped, 1: the singular values must be computed).
void launch_shrink_cert(symrom_rom& r) {
  const double tol = r.cfg.rank_tol_down;
  const double c = std::max(2.0 * tol * tol, 1e-13);
  launch_dense_rank_cert(r.s, r.Z0, r.n, r.p, c, r.status + 13);
}

// The end of a step: the tangent velocity Y(xi_half, Z_G) from the basis
// velocity in Xv (Sec. 5), xi_1 = dt Y, and U1 = R_{U0}(xi_1) into Uh with
// the re-orthonormalisation applied to Z1.
void tangent_retract(symrom_rom& r) {
  hipStream_t s = r.s;
  const int n = r.n, N = r.N;
  const double dt = r.cfg.dt;
  bool gram_ready = false;
  if (4 * n <= 64) {
    // one Gram of [U0, xi, U_half, X] and one row combination (the
    // intermediate Ups is never formed)
    Timer t(FAM_BASIS, s);
    launch_gemm_ah_b(s, ml(r.U0, n, r.Xi, n, r.Uh, n, r.Xv, n), 4 * n,
                     ml(r.U0, n, r.Xi, n, r.Uh, n, r.Xv, n), 4 * n, false, N, r.nkb, r.gemm_part,
                     r.Gram);
    launch_dense_tangent(s, r.Gram, n, dt, r.M1, r.M2, r.M3, r.flags);
    // xi_1, and in the same pass the Gram of [U0, xi_1] for the retraction
    gram_ready = launch_rowgemm_gram(s, rt(r.Xv, r.M1, n, r.Xi, r.M2, n, r.U0, r.M3, n), N, n,
                                     r.P, r.gemm_part, (size_t)r.nkb * 64 * 64, r.Gram, r.U0, n);
    if (!gram_ready)
      launch_rowgemm(s, rt(r.Xv, r.M1, n, r.Xi, r.M2, n, r.U0, r.M3, n), N, n, r.P);
  } else {
    Timer t(FAM_BASIS, s);
    launch_gemm_ah_b(s, ml(r.U0, n, r.Xi, n), 2 * n, ml(r.Xv, n, r.Uh, n), 2 * n, false, N,
                     r.nkb, r.gemm_part, r.Gram);
    launch_dense_tangent1(s, r.Amat, r.Gram, n, r.M1, r.M2, r.M3, r.C0x, r.flags);
    launch_rowgemm(s, rt(r.Xv, r.M1, n, r.Xi, r.M2, n, r.U0, r.M3, n), N, n, r.Ups);
    launch_gemm_ah_b(s, ml(r.Uh, n, r.U0, n), 2 * n, ml(r.Ups, n), n, false, N, r.nkb,
                     r.gemm_part, r.Gram);
    launch_dense_tangent2(s, r.Gram, r.C0x, n, dt, r.M1, r.M2, r.flags);
    launch_rowgemm(s, rt(r.Ups, r.M1, n, r.U0, r.M2, n), N, n, r.P);  // xi_1 = dt Y
  }
  // U1 = R_{U0}(xi_1)  (into Uh, free now)
  if (r.cfg.reorth && 4 * n <= 64) {
    cayley_cholqr2(r, r.U0, r.P, r.Uh, r.M3, r.Z1, gram_ready);
  } else {
    cayley(r, r.U0, r.P, r.Uh, r.M3, gram_ready);
    if (r.cfg.reorth) cholqr2(r, r.Uh, r.Z1);
  }
}

// One step of the reduced model; with decide_rank, the rank indicator at the
// new state and a growth by one pair when it exceeds the threshold.
symrom_status rom_step_one(symrom_rom& r, bool decide_rank) {
  hipStream_t s = r.s;
  const int n = r.n, p = r.p, N = r.N;
  const double dt = r.cfg.dt;
  // (word 3 belongs to a head that may be running on the second stream)
  HIPCHK(hipMemsetAsync(r.flags, 0, 3 * sizeof(int), s));
  const bool use_deim = r.cfg.projection == SYMROM_DEIM;
  // DMD-DEIM before its windows are full (Alg. 2, first T steps): the plain
  // reduced step, recording the snapshot and the subset potentials
  const bool record = r.cfg.projection == SYMROM_DMD_DEIM;
  // stage 1 at (U0, Z0): full gradient, k1 = J g, basis velocity -> xi_half.
  // With the fused gradient the Grams of U0 (its velocity part; also the
  // DEIM start's) are formed first, or were formed with the cached gradient.
  const bool fused = fused_gradient_ok(n);
  if (!r.stage1_cached) {
    if (fused) linear_grams(r, r.U0, r.C12a);
    full_gradient(r, r.U0, r.Z0, nullptr, true, false, nullptr, fused ? r.C12a : nullptr);
  }
  r.stage1_cached = false;
  // the DEIM chain is already enqueued when it was built ahead for this rank
  const bool chain_ready = use_deim && r.head_pending && r.head_n == n;
  if ((use_deim && !chain_ready) || record) {
    // the DEIM chain needs the first-stage field; it runs beside the basis
    // velocity, the Gram matrices of the linear part and the Cayley map
    HIPCHK(hipEventRecord(r.ev_fork, s));
    HIPCHK(hipStreamWaitEvent(r.s2, r.ev_fork, 0));
    deim_update(r, r.U0, r.Z0, r.head_pending);
  }
  r.head_pending = false;
  const bool deim = use_deim && r.deim_on;
  // (the eigensolver keeps one CU busy for a while: enqueue part of the main
  // work before the rest of the chain, so that both streams have work)
  basis_velocity(r, r.U0, r.Z0, 0.5 * dt, r.Xi, deim ? nullptr : r.k);
  if ((use_deim && !chain_ready) || record) {
    deim_update_tail(r);
    HIPCHK(hipEventRecord(r.ev_join, r.s2));
  }
  if (deim && !fused) linear_grams(r, r.U0, r.C12a);
  // U_half = R_{U0}(xi_half)
  cayley(r, r.U0, r.Xi, r.Uh, r.Amat);
  if (deim || fused) linear_grams(r, r.Uh, r.C12);
  if (use_deim || record) HIPCHK(hipStreamWaitEvent(s, r.ev_join, 0));
  // fixed point for k2 at U_half: start values (with DEIM in the launch that
  // gathers the first stage's gradient)
  if (deim) {
    Timer t(FAM_DENSE, s);
    const DeimStartArgs st{r.C12a, r.k, r.Zev, 0.5 * dt, r.prev, r.active, r.counters};
    launch_deim_gather(s, r.U0, N, n, r.Z0, p, r.Nx, r.b.factor, r.b.e, r.cfg.q / r.cfg.m, r.didx,
                       r.dw, r.d_cur, nullptr, r.gF, nullptr, &st);
  } else {
    Timer t(FAM_DENSE, s);
    launch_fp_init(s, r.prev, r.active, r.counters, p);
    launch_dense_finish_z(s, r.Z0, r.k, n, p, 0.5 * dt, r.Zev);
  }
  // The iterations are enqueued in batches with one counter readback per
  // batch: the first batch as long as the previous step's fixed point, then
  // one at a time.  Every launch in the loop is gated on the device counter
  // of active columns, so iterations enqueued past convergence do nothing
  // (and are not counted).  With kernel timing on, batches are single
  // iterations so that the work accounted to each launch is exact.
  const int fixed = r.cfg.fp_fixed_iters;
  const int limit = fixed > 0 ? fixed : r.cfg.fp_max_iters;
  const int* gate = r.counters;
  int hc[4] = {p, 0, 0, 0};
  r.n_active = p;
  int batch = fixed > 0 ? fixed : std::max(1, std::min(r.fp_hint, limit));
  if (g_timing) batch = 1;
  int launched = 0;
  while (launched < limit) {
    for (int b = 0; b < batch && launched < limit; ++b, ++launched) {
      if (deim) {
        const double pact = (double)r.n_active;
        {
          Timer t(FAM_DEPOSIT, s, 4.0 * n * (double)N * pact,
                  16.0 * n * ((double)N + p) + 8.0 * pact * r.Nx);
          launch_deposit_rom(s, r.Uh, N, n, r.Zev, p, r.Nx, r.gdep, r.b.factor, r.active,
                             r.b.part, gate, nullptr, r.cfg.deterministic);
        }
        {
          // per parameter: the Poisson solve, the DEIM gather of the sampled
          // rows and the fixed-point update of the column
          Timer t(FAM_POISSON, s);
          launch_poisson_deim(s, r.b.part, r.gdep.nrb, p, r.Nx, r.b.qw, r.b.h, r.b.mw, r.active,
                              r.b.rho, r.b.phi, r.b.e, r.b.energy, gate, r.Uh, N, n, r.Zev,
                              r.b.factor, r.cfg.q / r.cfg.m, r.didx, r.dw, r.d_cur, r.gF, r.C12,
                              r.Z0, r.ZG, r.k, r.prev, dt, r.cfg.fp_tol, r.cfg.fp_stall_tol,
                              fixed > 0 ? 1 : 0, launched + 1, r.counters);
        }
      } else {
        full_gradient(r, r.Uh, r.Zev, r.active, true, false, gate, fused ? r.C12 : nullptr);
        Timer t(FAM_DENSE, s);
        launch_dense_fp_update(s, r.gproj, r.C12, n, p, r.Z0, r.Zev, r.ZG, r.k, r.prev, r.active,
                               dt, r.cfg.fp_tol, r.cfg.fp_stall_tol, fixed > 0 ? 1 : 0, 0,
                               launched + 1, r.counters);
      }
    }
    LAUNCHCHK();
    // counters [0..2] and the largest stall-accepted update (words 6..7)
    HIPCHK(hipMemcpyAsync(r.hstat + 4, r.counters, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int q = 0; q < 3; ++q) hc[q] = r.hstat[4 + q];
    r.n_active = hc[0];
    if (hc[0] == 0) break;
    batch = 1;
  }
  const int iters = hc[2];
  if (fixed == 0) r.fp_hint = iters;
  r.last.iters = iters;
  r.last.stalled = hc[1];
  std::memcpy(&r.last.stall_rel, r.hstat + 10, sizeof(double));
  r.last.deim_active = deim ? 1 : 0;
  r.last.shrunk = 0;
  r.last.unconverged = 0;
  r.last.worst_rel = 0.0;
  if (fixed == 0 && hc[0] > 0) {
    // report the columns left and their last relative update
    {
      std::vector<int> act(p);
      std::vector<double> pv(p);
      if (hipMemcpy(act.data(), r.active, p * sizeof(int), hipMemcpyDeviceToHost) == hipSuccess &&
          hipMemcpy(pv.data(), r.prev, p * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess) {
        for (int i = 0; i < p; ++i)
          if (act[i]) {
            r.last.unconverged++;
            r.last.worst_rel = std::max(r.last.worst_rel, pv[i]);
          }
      }
    }
    // the state, the DEIM snapshot window included, stays as it was: the
    // snapshot of this step (counted in win_count whether it was taken now
    // or ahead of the step, and written into the slot of the oldest one,
    // which the next attempt at this step drops again) is taken back
    if (use_deim || record) {
      r.win_count--;
      r.deim_on = r.win_count >= r.nslots;
    }
    return fail(SYMROM_ENOCONV, "fixed point not converged");
  }
  // basis velocity at (U_half, Z_G) with the field of each column's last
  // evaluation; S(Z_G)^+ and Z1 = Z0 + dt k on the second stream (idle here)
  // beside the projection
  const bool side = r.s2 != nullptr;
  if (side) {
    HIPCHK(hipEventRecord(r.ev_sp0, s));
    HIPCHK(hipStreamWaitEvent(r.s2, r.ev_sp0, 0));
    Timer t(FAM_DENSE, r.s2);
    launch_dense_spinv(r.s2, r.ZG, n, p, r.cfg.pinv_rtol, r.Q, r.sigma2, r.flags);
    launch_dense_finish_z(r.s2, r.Z0, r.k, n, p, dt, r.Z1);
    HIPCHK(hipEventRecord(r.ev_sp1, r.s2));
  } else {
    launch_dense_finish_z(s, r.Z0, r.k, n, p, dt, r.Z1);
  }
  full_gradient(r, r.Uh, r.ZG, nullptr, false, false, nullptr, fused ? r.C12 : nullptr);
  if (side) HIPCHK(hipStreamWaitEvent(s, r.ev_sp1, 0));
  basis_velocity(r, r.Uh, r.ZG, 1.0, r.Xv, nullptr, side);
  if (r.split_U) {
    // the midpoint basis and the new coefficients, before the retraction
    // overwrites the one and rotates the other
    HIPCHK(hipMemcpyAsync(r.split_U, r.Uh, (size_t)N * n * sizeof(cplx), hipMemcpyDeviceToDevice,
                          s));
    HIPCHK(hipMemcpyAsync(r.split_Z, r.Z1, (size_t)n * p * sizeof(cplx), hipMemcpyDeviceToDevice,
                          s));
  }
  tangent_retract(r);
  // Commit by exchanging buffers before the flags are known, and with rank
  // adaptation enqueue the indicator's gradient at the new state behind it,
  // so that one readback serves both; a failed step exchanges them back.
  std::swap(r.U0, r.Uh);
  std::swap(r.Z0, r.Z1);
  // (the step's error words are final here)
  const bool ahead = use_deim && decide_rank;
  if ((use_deim || record) && !decide_rank) launch_fold_status(s, r.status);
  if (decide_rank) {
    // the field at the new state (its deposit also does the status
    // bookkeeping with DEIM), then (beside the DEIM chain ahead, which needs
    // only the field) its projection and the indicator
    full_gradient_field(r, r.U0, r.Z0, nullptr, nullptr, use_deim ? r.status : nullptr);
    if (ahead) HIPCHK(hipEventRecord(r.ev_fork, s));
    // (the Grams of the new U0 stay in C12a for the next step's first stage)
    if (fused) linear_grams(r, r.U0, r.C12a);
    full_gradient(r, r.U0, r.Z0, nullptr, false, true, nullptr, fused ? r.C12a : nullptr);
    launch_dense_indicator(s, r.colsq, r.gproj, n, p, r.eps_dev);
    if (r.cfg.rank_tol_down > 0.0) launch_shrink_cert(r);
  }
  // the status copy is started before the chain ahead is enqueued, and
  // waited for after
  HIPCHK(hipMemcpyAsync(r.hstat, r.status, 14 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(r.ev_read, s));
  if (ahead) {
    // the next step's DEIM chain, beside the readback; its head does
    // nothing if this step failed (stop word)
    HIPCHK(hipStreamWaitEvent(r.s2, r.ev_fork, 0));
    deim_update(r, r.U0, r.Z0, false, r.status + 12);
    deim_update_tail(r);
    HIPCHK(hipEventRecord(r.ev_join, r.s2));
    r.head_pending = true;
    r.head_n = n;
  }
  LAUNCHCHK();
  HIPCHK(hipEventSynchronize(r.ev_read));
  const int fl0 = r.hstat[0] | r.hstat[2];
  double eps = 0.0;
  std::memcpy(&eps, r.hstat + 8, sizeof(double));
  if (fl0) {
    std::swap(r.U0, r.Uh);
    std::swap(r.Z0, r.Z1);
    if (ahead) {
      // the head was gated off (the rest of the chain only rewrote the
      // operator, which the next step builds afresh)
      HIPCHK(hipStreamSynchronize(r.s2));
      r.head_pending = false;
      r.win_count--;
      r.deim_on = r.win_count >= r.nslots;
    }
    if (record) r.win_count--;  // the recorded level is taken back
    return fail(SYMROM_ESINGULAR, "singular small matrix in the basis update");
  }
  r.step++;
  if (!decide_rank) return SYMROM_OK;
  r.last.rank_indicator = eps;
  if (!(eps > r.cfg.rank_tol_up) || 2 * (n + 1) > r.cfg.two_n_max) {
    // the gradient just computed is the next step's first-stage gradient
    r.stage1_cached = true;
    // no growth: the automatic shrink, when the certificate does not rule it out
    if (r.cfg.rank_tol_down > 0.0 && r.hstat[13] != 0) return shrink_exact(r);
    return SYMROM_OK;
  }
  // the growth rewrites Z0 in its new layout: the head must be done with it
  if (r.head_pending) HIPCHK(hipStreamSynchronize(r.s2));
  HIPCHK(hipMemsetAsync(r.flags, 0, 2 * sizeof(int), s));
  return rom_grow_apply(r, 1);
}

// The handle's per-parameter buffers and sizes made those of the compact
// subset S (Sec. 4.1) for the exact gradient of the basis evolution; the
// whole ensemble is restored at the end of the scope.
struct SubsetView {
  symrom_rom& r;
  int p;
  PicBufs b;
  PicGeom gdep, ggat;
  int* sub;
  explicit SubsetView(symrom_rom& rr)
      : r(rr), p(rr.p), b(rr.b), gdep(rr.gdep), ggat(rr.ggat), sub(rr.sub) {
    r.p = r.psub;
    r.b = r.bs;
    r.gdep = r.gdep_s;
    r.ggat = r.ggat_s;
    r.sub = r.sub_id;
    r.n_active = r.psub;
  }
  ~SubsetView() {
    r.p = p;
    r.b = b;
    r.gdep = gdep;
    r.ggat = ggat;
    r.sub = sub;
    r.n_active = p;
  }
};

// One step of Alg. 2 once the windows hold T+1 levels (Sec. 4.3, eq.
// UZredhyp; the scheme of Sec. 5):
//   stage 1: the exact gradient of the subset at (U0, Z0[S]) gives the
//     snapshot and potential level of this step and k^1 = X(U0, Z0[S]);
//     U_half = R_{U0}(dt/2 k^1);
//   second stream: DEIM operator (snapshot Gram, Psi, indices, weights) and
//     DMD of the potential window, then the predicted field tables of every
//     parameter at t_{tau-1} and t_{tau-1} + dt/2;
//   the fixed point of every column with the DMD-DEIM gradient (one launch,
//     no deposit over the particles);
//   stage 2: the exact gradient of the subset at (U_half, Z_G[S]), the basis
//     velocity, the tangent velocity and the retraction with the
//     re-orthonormalisation of U1 and Z1 = Z0 + dt k.
// One readback per step: the error words and the fixed-point counters.
symrom_status rom_step_dmd(symrom_rom& r) {
  hipStream_t s = r.s;
  const int n = r.n, p = r.p, N = r.N, ps = r.psub;
  const double dt = r.cfg.dt;
  if (!r.beta_ready)
    return fail(SYMROM_ESTATE, "rom_step: DMD-DEIM needs the parameters (rom_set_parameters)");
  HIPCHK(hipMemsetAsync(r.flags, 0, 3 * sizeof(int), s));
  // counters: columns left, stalled, iterations, stall maximum; the DMD
  // chain's error word
  HIPCHK(hipMemsetAsync(r.counters, 0, 8 * sizeof(int), s));
  HIPCHK(hipMemsetAsync(r.status + 14, 0, sizeof(int), s));
  launch_gather_zcols(s, r.Z0, n, r.sub, ps, r.Zs);
  linear_grams(r, r.U0, r.C12a);
  {
    SubsetView v(r);
    full_gradient(r, r.U0, r.Zs, nullptr, true, false, nullptr, r.C12a);
    HIPCHK(hipEventRecord(r.ev_fork, s));
    HIPCHK(hipStreamWaitEvent(r.s2, r.ev_fork, 0));
    HIPCHK(hipStreamWaitEvent(r.s3, r.ev_fork, 0));
    deim_update(r, r.U0, r.Zs, false, nullptr, false);
    // this level's subset potentials into the window, on the DMD stream
    launch_grid_rows(r.s3, r.b.phi, nullptr, ps, r.Nx,
                     r.phiw + (size_t)((r.win_count - 1) % r.nslots) * ps * r.Nx);
    basis_velocity(r, r.U0, r.Zs, 0.5 * dt, r.Xi, nullptr);
  }
  deim_update_tail(r);
  HIPCHK(hipEventRecord(r.ev_join, r.s2));
  {
    // the DMD of the window (levels win_count - nslots .. win_count - 1)
    Timer t(FAM_DMD, r.s3);
    DmdChainArgs c = r.dmd;
    c.ring = r.phiw;
    c.nslots = r.nslots;
    c.base = r.win_count % r.nslots;
    c.pstar = ps;
    c.T = r.cfg.deim_window;
    c.Nx = r.Nx;
    c.tol = r.cfg.dmd_tol > 0.0 ? r.cfg.dmd_tol : 1e-5;
    // (its own error word, status word 14)
    c.flags = r.status + 14;
    launch_dmd_operator(r.s3, c);
    launch_dmd_tables(r.s3, c, p, r.beta, r.b.h, r.e0, r.eh);
  }
  HIPCHK(hipEventRecord(r.ev_join3, r.s3));
  cayley(r, r.U0, r.Xi, r.Uh, r.Amat);
  linear_grams(r, r.Uh, r.C12);
  HIPCHK(hipStreamWaitEvent(s, r.ev_join, 0));
  HIPCHK(hipStreamWaitEvent(s, r.ev_join3, 0));
  {
    const int fixed = r.cfg.fp_fixed_iters;
    Timer t(FAM_DMDFP, s);
    DmdFpArgs a{};
    a.U0 = r.U0;
    a.Uh = r.Uh;
    a.N = N;
    a.n = n;
    a.idx = r.didx;
    a.w = r.dw;
    a.d = r.d_cur;
    a.Z0 = r.Z0;
    a.factor = r.b.factor;
    a.e0 = r.e0;
    a.eh = r.eh;
    a.Nx = r.Nx;
    a.qm = r.cfg.q / r.cfg.m;
    a.C12a = r.C12a;
    a.C12 = r.C12;
    a.dt = dt;
    a.tol = r.cfg.fp_tol;
    a.stall_tol = r.cfg.fp_stall_tol;
    a.max_iters = r.cfg.fp_max_iters;
    a.fixed = fixed > 0 ? fixed : 0;
    a.k = r.k;
    a.ZG = r.ZG;
    a.prev = r.prev;
    a.active = r.active;
    a.counters = r.counters;
    launch_dmd_fp(s, a, p);
  }
  {
    Timer t(FAM_DENSE, s);
    launch_dense_finish_z(s, r.Z0, r.k, n, p, dt, r.Z1);
  }
  // stage 2: the subset's exact gradient at (U_half, Z_G[S]) and its basis velocity
  launch_gather_zcols(s, r.ZG, n, r.sub, ps, r.Zs);
  {
    SubsetView v(r);
    full_gradient(r, r.Uh, r.Zs, nullptr, true, false, nullptr, r.C12);
    basis_velocity(r, r.Uh, r.Zs, 1.0, r.Xv, nullptr);
  }
  if (r.split_U) {
    HIPCHK(hipMemcpyAsync(r.split_U, r.Uh, (size_t)N * n * sizeof(cplx), hipMemcpyDeviceToDevice,
                          s));
    HIPCHK(hipMemcpyAsync(r.split_Z, r.Z1, (size_t)n * p * sizeof(cplx), hipMemcpyDeviceToDevice,
                          s));
  }
  tangent_retract(r);
  std::swap(r.U0, r.Uh);
  std::swap(r.Z0, r.Z1);
  launch_fold_status(s, r.status);
  HIPCHK(hipMemcpyAsync(r.hstat, r.status, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  const int fl0 = r.hstat[0] | r.hstat[2] | r.hstat[14];
  r.last.iters = r.hstat[6];
  r.last.stalled = r.hstat[5];
  std::memcpy(&r.last.stall_rel, r.hstat + 10, sizeof(double));
  r.last.deim_active = 1;
  r.last.shrunk = 0;
  r.last.unconverged = 0;
  r.last.worst_rel = 0.0;
  if (r.hstat[4] > 0 || fl0) {
    std::swap(r.U0, r.Uh);
    std::swap(r.Z0, r.Z1);
    r.win_count--;
    r.deim_on = r.win_count >= r.nslots;
    if (fl0) {
      // error bits: 64 interpolation matrix, 128 SVD of the window, 256 QR
      // iteration of A_tol, 512 B rank deficient, others the basis update
      char msg[96];
      std::snprintf(msg, sizeof msg, "singular small matrix in the DMD-DEIM step (error bits 0x%x)",
                    (unsigned)fl0);
      return fail(SYMROM_ESINGULAR, msg);
    }
    std::vector<int> act(p);
    std::vector<double> pv(p);
    if (hipMemcpy(act.data(), r.active, p * sizeof(int), hipMemcpyDeviceToHost) == hipSuccess &&
        hipMemcpy(pv.data(), r.prev, p * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess) {
      for (int i = 0; i < p; ++i)
        if (act[i]) {
          r.last.unconverged++;
          r.last.worst_rel = std::max(r.last.worst_rel, pv[i]);
        }
    }
    return fail(SYMROM_ENOCONV, "fixed point not converged");
  }
  r.step++;
  return SYMROM_OK;
}
}  // namespace

extern "C" size_t rom_workspace_bytes(const symrom_config* cfg) {
  std::string why;
  if (!valid_rom_config(cfg, why)) return 0;
  symrom_rom r{};
  r.cfg = *cfg;
  r.N = cfg->N;
  r.p = cfg->p;
  r.Nx = cfg->Nx;
  r.nmax = cfg->two_n_max / 2;
  Arena ar(nullptr);
  carve_rom(ar, r);
  return ar.off + 256;
}

namespace {
symrom_status rom_upload_consts(symrom_rom& r, const double* L) {
  std::vector<int> sub(r.psub);
  for (int k = 0; k < r.psub; ++k) sub[k] = (int)(((long long)k * r.p) / r.psub);
  HIPCHK(hipMemcpyAsync(r.sub, sub.data(), r.psub * sizeof(int), hipMemcpyHostToDevice, r.s));
  r.win_count = 0;
  r.deim_on = false;
  std::vector<double> factor, qw, h, mw;
  per_param_consts(L, r.N, r.p, r.Nx, r.cfg.q, r.cfg.m, factor, qw, h, mw);
  hipStream_t s = r.s;
  HIPCHK(hipMemcpyAsync(r.b.factor, factor.data(), r.p * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(r.b.qw, qw.data(), r.p * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(r.b.h, h.data(), r.p * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(r.b.mw, mw.data(), r.p * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return SYMROM_OK;
}

// scale columns: M[:, c] = V[:, c] / sqrt(lam[c]) for c < r (p x r)
__global__ void scale_cols_kernel(const cplx* V, const double* lam, int p, int r, cplx* M) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= p * r) return;
  int c = t / p;
  M[t] = cscale(V[t], 1.0 / sqrt(lam[c]));
}

__global__ void scale_col_kernel(cplx* u, int N, double sc) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < N) u[l] = cscale(u[l], sc);
}

// column c of U <- e_j - U[:, :c] conj(U[j, :c])^T  (Gram-Schmidt of e_j)
__global__ void unit_minus_proj_kernel(cplx* U, int N, int c, int j) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= N) return;
  cplx v = mk(l == j ? 1.0 : 0.0, 0.0);
  for (int k = 0; k < c; ++k) {
    cplx ujk = U[(size_t)k * N + j];
    v = csub(v, cmulc(ujk, U[(size_t)k * N + l]));  // conj(U[j,k]) U[l,k]
  }
  U[(size_t)c * N + l] = v;
}
}  // namespace

namespace {
// Gram G = A^* A (p x p, ld p) of an N x p matrix with p > 64: the blocks of
// 64 columns on and above the diagonal by the split-K product, each placed
// with its conjugate transpose.
void gram_big(symrom_rom& r, const cplx* A, int p, cplx* G) {
  hipStream_t s = r.s;
  const size_t N = (size_t)r.N;
  for (int a0 = 0; a0 < p; a0 += 64) {
    const int ac = std::min(64, p - a0);
    for (int b0 = a0; b0 < p; b0 += 64) {
      const int bc = std::min(64, p - b0);
      launch_gemm_ah_b(s, ml(A + a0 * N, ac), ac, ml(A + b0 * N, bc), bc, false, r.N, r.nkb,
                       r.gemm_part, r.Gram);
      launch_scatter_block(s, r.Gram, ac, bc, G, p, a0, b0);
    }
  }
}

// The k leading eigenpairs of a Hermitian p x p matrix A (p > 64, k <= 48)
// by subspace iteration with Rayleigh-Ritz on m = min(k + 16, 64) vectors:
// W = orth(A V); H = W^* A W (m x m); V = W Y with H = Y diag(lam) Y^*
// (decreasing).  The leading k Ritz values settle first; the iteration then
// runs on until the subspace angle, which shrinks by rho = lam_m / lam_k per
// iteration, is below 1e-15 of its value at that point times 1e-8 (about
// the square root of the Ritz-value tolerance).  V: p x m (ld p), W: p x m
// scratch; lam (m, device) and the count m.  At most 400 iterations.
symrom_status topeig_subspace(symrom_rom& r, const cplx* A, int p, int k, cplx* V, cplx* W,
                              double* lam, int* m_out) {
  hipStream_t s = r.s;
  const int m = std::min(64, std::min(p, k + 16));
  std::vector<cplx> v0((size_t)p * m);
  uint64_t x = 0x9e3779b97f4a7c15ull;
  for (auto& v : v0) {
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    const double a = (double)(x >> 11) * 0x1p-53 - 0.5;
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    const double b = (double)(x >> 11) * 0x1p-53 - 0.5;
    v = mk(a, b);
  }
  HIPCHK(hipMemcpyAsync(V, v0.data(), v0.size() * sizeof(cplx), hipMemcpyHostToDevice, s));
  launch_cgs2(s, V, p, m);
  std::vector<double> prev(m, 0.0), cur(m);
  int extra = -1;  // iterations still to run once the Ritz values settled
  for (int it = 0; it < 400; ++it) {
    launch_herm_mm(s, A, V, p, m, W);
    launch_cgs2(s, W, p, m);
    launch_herm_mm(s, A, W, p, m, V);
    launch_gemm_ah_b(s, ml(W, m), m, ml(V, m), m, false, p, r.nkb, r.gemm_part, r.Gram);
    launch_dense_herm_eig(s, r.Gram, m, r.Ysub, lam, r.flags);
    launch_rowgemm(s, rt(W, r.Ysub, m), p, m, V);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(cur.data(), lam, m * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (extra > 0) {
      if (--extra == 0) break;
    } else if (it >= 2) {
      double dmax = 0.0;
      for (int j = 0; j < k; ++j) dmax = std::max(dmax, std::fabs(cur[j] - prev[j]));
      if (dmax <= 1e-14 * std::fabs(cur[0])) {
        const double rho = (cur[k - 1] > 0.0) ? std::fabs(cur[m - 1]) / cur[k - 1] : 1.0;
        extra = (rho < 1e-3) ? 3 : std::min(300, 3 + (int)std::ceil(std::log(1e-8) / std::log(rho)));
      }
    }
    prev = cur;
  }
  *m_out = m;
  return SYMROM_OK;
}
}  // namespace

namespace {
// fill(r): writes C0 = X0 + i V0 into r.G on r.s
symrom_status set_parameters(symrom_rom& r, const double* eta, int dim);

symrom_status rom_init_impl(const symrom_config* cfg, const double* L,
                            const std::function<bool(symrom_rom&)>& fill, const double* eta4,
                            void* ws, size_t ws_bytes, void* stream, symrom_rom** out) {
  std::string why;
  if (!valid_rom_config(cfg, why)) return fail(SYMROM_EINVAL, "rom_init: " + why);
  if (!L || !out) return fail(SYMROM_EINVAL, "rom_init: null pointer");
  for (int i = 0; i < cfg->p; ++i)
    if (!(L[i] > 0.0) || !std::isfinite(L[i])) return fail(SYMROM_EINVAL, "rom_init: bad L");
  // the DMD of the potential treats the potentials of all parameters as
  // vectors on one grid (Sec. 4.2.1: the potential depends on the parameter
  // only through the state)
  if (cfg->projection == SYMROM_DMD_DEIM)
    for (int i = 1; i < cfg->p; ++i)
      if (L[i] != L[0]) return fail(SYMROM_EINVAL, "rom_init: DMD-DEIM needs one domain length");
  size_t need = rom_workspace_bytes(cfg);
  if (!ws || ws_bytes < need) return fail(SYMROM_ENOMEM, "rom_init: workspace too small");
  symrom_rom* r = new symrom_rom{};
  r->cfg = *cfg;
  if (r->cfg.fp_stall_tol == 0.0) r->cfg.fp_stall_tol = 1e-3;
  r->N = cfg->N;
  r->p = cfg->p;
  r->Nx = cfg->Nx;
  r->n = cfg->two_n / 2;
  r->nmax = cfg->two_n_max / 2;
  r->s = (hipStream_t)stream;
  r->last.rank_indicator = -1.0;
  Arena ar(ws);
  carve_rom(ar, *r);
  symrom_status st = rom_upload_consts(*r, L);
  if (st != SYMROM_OK) {
    delete r;
    return st;
  }
  hipStream_t s = r->s;
  const int N = r->N, p = r->p, n = r->n;
  if (hipMemsetAsync(r->status, 0, 16 * sizeof(int), s) != hipSuccess) {
    delete r;
    return fail(SYMROM_EDEVICE, "rom_init: memset");
  }
  // C0 = X0 + i V0 in the gather buffer; Gram C0^* C0 (p x p) and its
  // leading eigenpairs: all of them by Jacobi for p <= 64, the leading ones
  // by subspace iteration beyond
  if (!fill(*r)) {
    delete r;
    return fail(SYMROM_EDEVICE, "rom_init: initial state");
  }
  int nl = p;
  if (p <= 64) {
    launch_gemm_ah_b(s, ml(r->G, p), p, ml(r->G, p), p, false, N, r->nkb, r->gemm_part, r->Gp);
    launch_dense_herm_eig(s, r->Gp, p, r->Vp, r->lam, r->flags);
  } else {
    gram_big(*r, r->G, p, r->Gp);
    symrom_status st2 = topeig_subspace(*r, r->Gp, p, n, r->Vp, r->Wsub, r->lam, &nl);
    if (st2 != SYMROM_OK) {
      delete r;
      return st2;
    }
  }
  std::vector<double> lam(nl);
  if (hipMemcpyAsync(lam.data(), r->lam, nl * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    delete r;
    return fail(SYMROM_EDEVICE, "rom_init: eigen readback");
  }
  // the singular values of C0 (all p by Jacobi; the n converged leading ones
  // of the subspace iteration beyond 64)
  {
    const int ns = (p <= 64) ? nl : std::min(nl, n);
    r->init_sig.resize(ns);
    for (int j = 0; j < ns; ++j) r->init_sig[j] = std::sqrt(std::max(lam[j], 0.0));
  }
  // The basis: the leading eigenpairs of C0^* C0 (U = C0 V lam^{-1/2}),
  // completed by Gram-Schmidt of e_0, e_1, ..., then two Cholesky-QR passes
  // and Z = U^* C0.  Eigenpairs far below the largest are not resolved by
  // the Gram (their vectors are rounding): when the orthonormalisation fails
  // with every pair above 1e-26 lam_0, it is redone with the pairs above
  // 1e-13 lam_0 (vectors accurate to about 1e-3, which the Cholesky-QR
  // passes repair), the completion taking the rest.
  const double lam_floor[2] = {1e-26, 1e-13};
  int fl[2] = {0, 0};
  int rk_prev = -1;
  for (int attempt = 0; attempt < 2; ++attempt) {
    int rk = 0;
    while (rk < n && rk < nl && lam[rk] > lam_floor[attempt] * lam[0] && lam[rk] > 0.0) ++rk;
    if (rk == rk_prev) break;
    rk_prev = rk;
    if (hipMemsetAsync(r->flags, 0, 2 * sizeof(int), s) != hipSuccess) {
      delete r;
      return fail(SYMROM_EDEVICE, "rom_init: memset");
    }
    // U[:, :rk] = C0 V_rk diag(lam)^{-1/2}
    hipLaunchKernelGGL(scale_cols_kernel, dim3((p * rk + 255) / 256 + 1), dim3(256), 0, s, r->Vp,
                       r->lam, p, rk, r->Q);
    if (rk > 0) launch_rowgemm(s, rt(r->G, r->Q, p), N, rk, r->U0);
    // completion by Gram-Schmidt of e_0, e_1, ... (two projections via CholQR2)
    int j = 0;
    int have = rk;
    std::vector<cplx> gram;
    while (have < n) {
      if (j >= N) {
        delete r;
        return fail(SYMROM_EINVAL, "rom_init: cannot complete the basis");
      }
      hipLaunchKernelGGL(unit_minus_proj_kernel, dim3((N + 255) / 256), dim3(256), 0, s, r->U0, N,
                         have, j);
      // accept if the projected vector is not negligible
      launch_gemm_ah_b(s, ml(r->U0 + (size_t)have * N, 1), 1, ml(r->U0 + (size_t)have * N, 1), 1,
                       false, N, r->nkb, r->gemm_part, r->Gram);
      cplx nv;
      if (hipMemcpyAsync(&nv, r->Gram, sizeof(cplx), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        delete r;
        return fail(SYMROM_EDEVICE, "rom_init: readback");
      }
      ++j;
      if (std::sqrt(nv.re) > 1e-8) {
        hipLaunchKernelGGL(scale_col_kernel, dim3((N + 255) / 256), dim3(256), 0, s,
                           r->U0 + (size_t)have * N, N, 1.0 / std::sqrt(nv.re));
        ++have;
      }
    }
    // orthonormalise (CholQR2), then Z = U^* C0
    r->n = n;
    launch_fill_cplx(s, r->Z0, (size_t)n * p, mk(0.0, 0.0));
    cholqr2(*r, r->U0, nullptr);
    launch_gemm_ah_b(s, ml(r->U0, n), n, ml(r->G, p), p, false, N, r->nkb, r->gemm_part, r->Z0);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      delete r;
      return fail(SYMROM_EDEVICE, "rom_init: launch failure");
    }
    if (hipMemcpy(fl, r->flags, 2 * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
      delete r;
      return fail(SYMROM_EDEVICE, "rom_init: flags readback");
    }
    if (!fl[0]) break;
  }
  if (fl[0]) {
    delete r;
    return fail(SYMROM_ESINGULAR, "rom_init: basis orthonormalisation failed");
  }
  if (hipHostMalloc((void**)&r->hstat, 64, hipHostMallocDefault) != hipSuccess) {
    r->hstat = nullptr;
    rom_destroy(r);
    return fail(SYMROM_EDEVICE, "rom_init: pinned status buffer");
  }
  if (hipEventCreateWithFlags(&r->ev_read, hipEventDisableTiming) != hipSuccess) {
    r->ev_read = nullptr;
    rom_destroy(r);
    return fail(SYMROM_EDEVICE, "rom_init: event creation");
  }
  if (cfg->projection != SYMROM_GALERKIN &&
      (hipStreamCreateWithFlags(&r->s2, hipStreamNonBlocking) != hipSuccess ||
       hipEventCreateWithFlags(&r->ev_fork, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&r->ev_join, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&r->ev_sp0, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&r->ev_sp1, hipEventDisableTiming) != hipSuccess)) {
    rom_destroy(r);
    return fail(SYMROM_EDEVICE, "rom_init: stream or event creation");
  }
  if (cfg->projection == SYMROM_DMD_DEIM &&
      (hipStreamCreateWithFlags(&r->s3, hipStreamNonBlocking) != hipSuccess ||
       hipEventCreateWithFlags(&r->ev_join3, hipEventDisableTiming) != hipSuccess)) {
    rom_destroy(r);
    return fail(SYMROM_EDEVICE, "rom_init: stream or event creation");
  }
  if (cfg->projection == SYMROM_DMD_DEIM) {
    // the parameter subset of eq. pSampl from Z^0, fixed from now on, and
    // the per-parameter constants of its compact columns
    const int ps = r->psub;
    launch_subset_select(s, r->Z0, n, p, ps, r->dmin, r->sub);
    std::vector<int> S(ps), id(ps);
    for (int k = 0; k < ps; ++k) id[k] = k;
    std::vector<double> Ls(ps), factor, qw, h, mw;
    // (no DMD yet: rank 0 until the first DMD-DEIM step)
    bool okc = hipMemsetAsync(r->dmd.rdev, 0, 4 * sizeof(int), s) == hipSuccess &&
               hipMemcpyAsync(S.data(), r->sub, ps * sizeof(int), hipMemcpyDeviceToHost, s) ==
                   hipSuccess &&
               hipMemcpyAsync(r->sub_id, id.data(), ps * sizeof(int), hipMemcpyHostToDevice, s) ==
                   hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    if (okc) {
      for (int k = 0; k < ps; ++k) Ls[k] = L[S[k]];
      per_param_consts(Ls.data(), N, ps, r->Nx, cfg->q, cfg->m, factor, qw, h, mw);
      okc = hipMemcpyAsync(r->bs.factor, factor.data(), ps * 8, hipMemcpyHostToDevice, s) ==
                hipSuccess &&
            hipMemcpyAsync(r->bs.qw, qw.data(), ps * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
            hipMemcpyAsync(r->bs.h, h.data(), ps * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
            hipMemcpyAsync(r->bs.mw, mw.data(), ps * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
            hipStreamSynchronize(s) == hipSuccess;
    }
    if (!okc) {
      rom_destroy(r);
      return fail(SYMROM_EDEVICE, "rom_init: parameter subset");
    }
    r->beta_ready = false;
    if (eta4) {
      r->ready = true;
      const symrom_status st2 = set_parameters(*r, eta4, 4);
      if (st2 != SYMROM_OK) {
        rom_destroy(r);
        return st2;
      }
    }
  }
  r->ready = true;
  r->stage1_cached = false;
  r->step = 0;
  *out = r;
  return SYMROM_OK;
}

// eta (host, dim per parameter) into the handle and the radial basis
// weights of the subset nodes (Sec. 4.2.1)
symrom_status set_parameters(symrom_rom& r, const double* eta, int dim) {
  hipStream_t s = r.s;
  for (int q = 0; q < r.p * dim; ++q)
    if (!std::isfinite(eta[q])) return fail(SYMROM_EINVAL, "rom_set_parameters: non-finite eta");
  HIPCHK(hipMemsetAsync(r.flags, 0, sizeof(int), s));
  HIPCHK(hipMemcpyAsync(r.eta, eta, (size_t)r.p * dim * sizeof(double), hipMemcpyHostToDevice, s));
  launch_rbf_weights(s, r.eta, dim, r.p, r.sub, r.psub, r.member, r.beta, r.flags);
  LAUNCHCHK();
  int fl = 0;
  HIPCHK(hipMemcpyAsync(&fl, r.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (fl & 64) return fail(SYMROM_ESINGULAR, "rom_set_parameters: interpolation matrix not positive definite");
  r.eta_dim = dim;
  r.beta_ready = true;
  return SYMROM_OK;
}
}  // namespace

extern "C" symrom_status rom_init(const symrom_config* cfg, const double* L, const double* X0,
                                  const double* V0, void* ws, size_t ws_bytes, void* stream,
                                  symrom_rom** out) {
  if (!X0 || !V0) return fail(SYMROM_EINVAL, "rom_init: null state");
  auto fill = [&](symrom_rom& r) {
    launch_make_complex(r.s, X0, V0, (size_t)r.N * r.p, r.G);
    return hipGetLastError() == hipSuccess;
  };
  return rom_init_impl(cfg, L, fill, nullptr, ws, ws_bytes, stream, out);
}

extern "C" symrom_status rom_init_family(const symrom_config* cfg, int32_t family,
                                         const double* eta, const double* ux, const double* uv,
                                         void* ws, size_t ws_bytes, void* stream,
                                         symrom_rom** out) {
  std::vector<double> L;
  if (!cfg || !eta || !ux || !uv || (family != 0 && family != 1) || cfg->p <= 0 ||
      !eta_lengths(cfg->p, eta, L))
    return fail(SYMROM_EINVAL, "rom_init_family: bad arguments");
  const int p = cfg->p;
  // eta is staged in the deposit-partials buffer (at least 32 p doubles),
  // which nothing uses before the first step
  auto fill = [&](symrom_rom& r) {
    if (hipMemcpyAsync(r.b.part, eta, (size_t)4 * p * sizeof(double), hipMemcpyHostToDevice,
                       r.s) != hipSuccess)
      return false;
    launch_load_family(r.s, family, r.N, p, r.b.part, ux, uv, nullptr, nullptr, r.G);
    return hipGetLastError() == hipSuccess;
  };
  return rom_init_impl(cfg, L.data(), fill, eta, ws, ws_bytes, stream, out);
}

extern "C" symrom_status symrom_load_family(int32_t family, int32_t N, int32_t p,
                                            const double* eta, const double* ux, const double* uv,
                                            double* X, double* V, void* stream) {
  if (N <= 0 || p <= 0 || !eta || !ux || !uv || (family != 0 && family != 1))
    return fail(SYMROM_EINVAL, "symrom_load_family: bad arguments");
  launch_load_family((hipStream_t)stream, family, N, p, eta, ux, uv, X, V, nullptr);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  return SYMROM_OK;
}

namespace {
symrom_status rom_grow(symrom_rom& r, int k, bool decide);

// Entry points other than rom_step first wait for a DEIM head enqueued
// ahead (it reads the state and the field buffers they may rewrite).
void side_wait(symrom_rom* r) {
  if (r && r->s2 && r->head_pending) (void)hipStreamSynchronize(r->s2);
}
}

extern "C" symrom_status rom_step(symrom_rom* r, int32_t nsteps, symrom_step_info* info) {
  if (!r || nsteps < 0) return fail(SYMROM_EINVAL, "rom_step: bad arguments");
  if (!r->ready) return fail(SYMROM_ESTATE, "rom_step: handle not initialised");
  int64_t iters_total = 0, deim_steps = 0, stalled_total = 0;
  double stall_max = 0.0;
  r->last.iters_total = 0;
  r->last.deim_steps = 0;
  r->last.stalled_total = 0;
  for (int it = 0; it < nsteps; ++it) {
    // DMD-DEIM (Alg. 2): the plain step until the windows hold T+1 levels
    const bool dmd = r->cfg.projection == SYMROM_DMD_DEIM && r->win_count + 1 >= r->nslots;
    symrom_status st = dmd ? rom_step_dmd(*r) : rom_step_one(*r, r->cfg.rank_auto != 0);
    iters_total += r->last.iters;
    deim_steps += r->last.deim_active;
    stalled_total += r->last.stalled;
    stall_max = std::max(stall_max, r->last.stall_rel);
    r->last.stall_rel = stall_max;
    r->last.iters_total = (int32_t)iters_total;
    r->last.deim_steps = (int32_t)deim_steps;
    r->last.stalled_total = (int32_t)stalled_total;
    if (st != SYMROM_OK) {
      r->last.two_n = 2 * r->n;
      if (info) *info = r->last;
      return st;
    }
  }
  r->last.two_n = 2 * r->n;
  if (info) *info = r->last;
  return SYMROM_OK;
}

namespace {
// Grow by k pairs (k > 0), or only evaluate the indicator when k == 0 and
// decide = true (then grow one pair if eps > rank_tol_up and the cap allows).
symrom_status rom_grow(symrom_rom& r, int k, bool decide) {
  hipStream_t s = r.s;
  const int n = r.n, p = r.p;
  HIPCHK(hipMemsetAsync(r.flags, 0, 2 * sizeof(int), s));
  // (the Grams of U0 into C12a: this gradient may become the next step's
  // first stage)
  const bool fused = fused_gradient_ok(n);
  if (fused) linear_grams(r, r.U0, r.C12a);
  full_gradient(r, r.U0, r.Z0, nullptr, true, decide, nullptr, fused ? r.C12a : nullptr);
  if (decide) {
    // eps needs only |G|^2 and |g|^2
    launch_dense_indicator(s, r.colsq, r.gproj, n, p, r.eps_dev);
    LAUNCHCHK();
    {
      symrom_status st = read_status(r);
      if (st != SYMROM_OK) return st;
    }
    double eps = 0.0;
    std::memcpy(&eps, r.hstat + 8, sizeof(double));
    r.last.rank_indicator = eps;
    if (!(eps > r.cfg.rank_tol_up) || 2 * (n + 1) > r.cfg.two_n_max) {
      // the gradient just computed is the next step's first-stage gradient
      r.stage1_cached = true;
      if (r.cfg.rank_tol_down > 0.0) {
        launch_shrink_cert(r);
        LAUNCHCHK();
        int word = 0;
        HIPCHK(hipMemcpyAsync(&word, r.status + 13, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (word != 0) return shrink_exact(r);
      }
      return SYMROM_OK;
    }
    k = 1;
  }
  return rom_grow_apply(r, k);
}

// The automatic shrink after the certificate failed: the singular values of
// Z~ (one-sided Jacobi), then a rotation to the singular vectors of Z~ and
// the drop of the pairs below rank_tol_down times the largest (at least one
// pair is kept).
symrom_status shrink_exact(symrom_rom& r) {
  hipStream_t s = r.s;
  const int n = r.n, p = r.p;
  cplx* work = (p >= n) ? r.Gp : r.Xv;
  launch_dense_zsvals(s, r.Z0, n, p, work, r.zsig);
  LAUNCHCHK();
  std::vector<double> sg(n);
  HIPCHK(hipMemcpyAsync(sg.data(), r.zsig, n * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (!(sg[0] > 0.0)) return SYMROM_OK;
  int keep = 0;
  for (int a = 0; a < n; ++a)
    if (sg[a] >= r.cfg.rank_tol_down * sg[0]) ++keep;
  if (keep < 1) keep = 1;
  if (keep >= n) return SYMROM_OK;
  // the DEIM head built ahead reads U0 and Z0; the next step builds it again
  if (r.head_pending && r.s2) HIPCHK(hipStreamSynchronize(r.s2));
  symrom_status st = rom_shrink(r, keep);
  r.stage1_cached = false;
  r.head_n = -1;
  r.last.shrunk = n - keep;
  return st;
}

// Growth by k pairs with the full gradient at (U0, Z0) (field and g) in the
// buffers; flags cleared by the caller.
symrom_status rom_grow_apply(symrom_rom& r, int k) {
  hipStream_t s = r.s;
  const int n = r.n, p = r.p, N = r.N;
  r.stage1_cached = false;
  if (n + k > r.nmax) return fail(SYMROM_ERANKCAP, "rank growth beyond two_n_max");
  if (k > p) return fail(SYMROM_EINVAL, "cannot grow by more pairs than parameters");
  if (fused_gradient_ok(n)) materialise_gradient(r, r.U0, r.Z0);
  if (p <= 64)
    launch_gemm_ah_b(s, ml(r.G, p), p, ml(r.G, p), p, false, N, r.nkb, r.gemm_part, r.Gp);
  else
    gram_big(r, r.G, p, r.Gp);
  launch_dense_hh(s, r.Gp, r.gproj, n, p, nullptr);
  LAUNCHCHK();
  if (p <= 64) {
    launch_dense_herm_eig(s, r.Gp, p, r.Vp, r.lam, r.flags);
  } else {
    int ml_ = 0;
    symrom_status st2 = topeig_subspace(r, r.Gp, p, k, r.Vp, r.Wsub, r.lam, &ml_);
    if (st2 != SYMROM_OK) return st2;
  }
  launch_dense_grow_prep(s, r.Vp, r.lam, r.gproj, n, p, k, r.Q, r.MP, r.flags);
  // the new columns go beyond the current basis (the state is not touched
  // until the flags are known)
  cplx* Y = r.U0 + (size_t)n * N;
  launch_rowgemm(s, rt(r.G, r.Q, p, r.U0, r.MP, n), N, k, Y);
  // Y came through the eigenvectors of a p x p Gram, so it is orthogonal to
  // U~ and orthonormal only to about eps cond^2: project U~ out of it and
  // orthonormalise it by Cholesky QR, twice (R = U Z is unaffected: the new
  // coefficient rows are zero)
  for (int pass = 0; pass < 2; ++pass) {
    launch_gemm_ah_b(s, ml(r.U0, n), n, ml(Y, k), k, false, N, r.nkb, r.gemm_part, r.M1);
    launch_proj_mats(s, r.M1, n, k, r.M2, r.M3);
    launch_rowgemm(s, rt(Y, r.M2, k, r.U0, r.M3, n), N, k, r.Xv);
    launch_copy_cplx(s, Y, r.Xv, (size_t)N * k);
    launch_gemm_ah_b(s, ml(Y, k), k, ml(Y, k), k, false, N, r.nkb, r.gemm_part, r.Gram);
    launch_cholqr_apply(s, r.Gram, k, Y, N, nullptr, p, r.flags);
  }
  launch_colphase(s, r.U0, N, n, k);
  LAUNCHCHK();
  int fl[2];
  symrom_status st = read_flags(r, fl);
  if (st != SYMROM_OK) return st;
  if (fl[0]) return fail(SYMROM_ESINGULAR, "rank growth: indicator matrix has too small rank");
  launch_z_resize(s, r.Z0, n, r.Z1, n + k, p);
  std::swap(r.Z0, r.Z1);
  LAUNCHCHK();
  r.n = n + k;
  r.head_n = -1;
  return SYMROM_OK;
}

symrom_status rom_shrink(symrom_rom& r, int n_new) {
  hipStream_t s = r.s;
  const int n = r.n, p = r.p, N = r.N;
  launch_dense_shrink(s, r.Z0, n, p, r.M1, r.Z1, r.sigma2);
  launch_rowgemm(s, rt(r.U0, r.M1, n), N, n_new, r.Uh);
  std::swap(r.U0, r.Uh);
  launch_z_resize(s, r.Z1, n, r.Z0, n_new, p);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  r.n = n_new;
  return SYMROM_OK;
}
}  // namespace

extern "C" symrom_status rom_adapt_rank(symrom_rom* r, int32_t target_two_n, int32_t* new_two_n) {
  side_wait(r);
  if (!r) return fail(SYMROM_EINVAL, "rom_adapt_rank: null handle");
  r->stage1_cached = false;
  if (!r->ready) return fail(SYMROM_ESTATE, "rom_adapt_rank: handle not initialised");
  if (target_two_n < 0 || (target_two_n & 1))
    return fail(SYMROM_EINVAL, "rom_adapt_rank: target must be even and non-negative");
  if (target_two_n > r->cfg.two_n_max) return fail(SYMROM_ERANKCAP, "rom_adapt_rank: above cap");
  symrom_status st = SYMROM_OK;
  r->last.shrunk = 0;
  const int n_before = r->n;
  if (target_two_n == 0)
    st = rom_grow(*r, 0, true);
  else if (target_two_n > 2 * r->n)
    st = rom_grow(*r, (target_two_n - 2 * r->n) / 2, false);
  else if (target_two_n < 2 * r->n)
    st = rom_shrink(*r, target_two_n / 2);
  // a DEIM head built ahead of the next step snapshots the state it saw:
  // after any change of U or Z it is rebuilt (same slot) by the next step
  if (target_two_n != 0 && target_two_n != 2 * n_before) r->head_n = -1;
  if (r->n != n_before) r->head_n = -1;
  if (new_two_n) *new_two_n = 2 * r->n;
  return st;
}

extern "C" symrom_status rom_get_state(symrom_rom* r, double* UX, double* Z, int32_t* two_n,
                                       int64_t* step) {
  side_wait(r);
  if (!r) return fail(SYMROM_EINVAL, "rom_get_state: null handle");
  hipStream_t s = r->s;
  if (UX) launch_ux_from_u(s, r->U0, r->N, r->n, UX);
  if (Z) launch_z_to_real(s, r->Z0, r->n, r->p, Z);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  if (two_n) *two_n = 2 * r->n;
  if (step) *step = r->step;
  return SYMROM_OK;
}

extern "C" symrom_status rom_set_state(symrom_rom* r, int32_t two_n, const double* UX,
                                       const double* Z, int64_t step) {
  side_wait(r);
  if (!r || !UX || !Z) return fail(SYMROM_EINVAL, "rom_set_state: null argument");
  if (two_n <= 0 || (two_n & 1) || two_n > r->cfg.two_n_max)
    return fail(SYMROM_EINVAL, "rom_set_state: bad rank");
  r->n = two_n / 2;
  r->stage1_cached = false;
  hipStream_t s = r->s;
  launch_u_from_ux(s, UX, r->N, r->n, r->U0);
  launch_z_from_real(s, Z, r->n, r->p, r->Z0);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  r->step = step;
  r->ready = true;
  r->win_count = 0;
  r->deim_on = false;
  r->head_pending = false;
  return SYMROM_OK;
}

extern "C" symrom_status rom_reconstruct(symrom_rom* r, double* X, double* V) {
  side_wait(r);
  if (!r) return fail(SYMROM_EINVAL, "rom_reconstruct: null handle");
  launch_reconstruct(r->s, r->U0, r->N, r->n, r->Z0, r->p, X, V);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(r->s));
  return SYMROM_OK;
}

extern "C" symrom_status rom_set_fixed_point(symrom_rom* r, double fp_tol, int32_t fp_max_iters,
                                             int32_t fp_fixed_iters) {
  if (!r || !(fp_tol >= 0.0) || fp_max_iters < 1 || fp_fixed_iters < 0)
    return fail(SYMROM_EINVAL, "rom_set_fixed_point: bad arguments");
  r->cfg.fp_tol = fp_tol;
  r->cfg.fp_max_iters = fp_max_iters;
  r->cfg.fp_fixed_iters = fp_fixed_iters;
  return SYMROM_OK;
}

extern "C" symrom_status rom_reconstruct_rows(symrom_rom* r, const int32_t* rows, int32_t nrows,
                                              double* X, double* V) {
  side_wait(r);
  if (!r || !rows || nrows < 0) return fail(SYMROM_EINVAL, "rom_reconstruct_rows: bad arguments");
  launch_reconstruct(r->s, r->U0, r->N, r->n, r->Z0, r->p, X, V, rows, nrows);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(r->s));
  return SYMROM_OK;
}

extern "C" symrom_status rom_cells(symrom_rom* r, const double* Z, int32_t* cells, double* s) {
  side_wait(r);
  if (!r || !cells) return fail(SYMROM_EINVAL, "rom_cells: null argument");
  hipStream_t st = r->s;
  const cplx* Zc = r->Z0;
  if (Z) {
    r->stage1_cached = false;
    launch_z_from_real(st, Z, r->n, r->p, r->Zev);
    Zc = r->Zev;
  }
  launch_rom_cells(st, r->U0, r->N, r->n, Zc, r->p, r->Nx, r->b.factor, cells, s);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));
  return SYMROM_OK;
}

extern "C" symrom_status rom_deim_operator(symrom_rom* r, int32_t* idx, double* w, int32_t* d) {
  side_wait(r);
  if (!r || !idx || !w) return fail(SYMROM_EINVAL, "rom_deim_operator: null argument");
  if (r->cfg.projection == SYMROM_GALERKIN || !r->deim_on)
    return fail(SYMROM_ESTATE, "rom_deim_operator: no DEIM operator has been built");
  hipStream_t s = r->s;
  HIPCHK(hipMemcpyAsync(idx, r->didx, r->d_cur * sizeof(int), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(w, r->dw, r->d_cur * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  if (d) *d = r->d_cur;
  return SYMROM_OK;
}

// ---------------------------------------------------------------------------
// stateless DEIM selection on a given basis (the kernels of the step)
// ---------------------------------------------------------------------------
extern "C" symrom_status rom_set_parameters(symrom_rom* r, const double* eta, int32_t dim) {
  if (!r || !eta || dim < 1 || dim > 8) return fail(SYMROM_EINVAL, "rom_set_parameters: bad arguments");
  if (!r->ready) return fail(SYMROM_ESTATE, "rom_set_parameters: handle not initialised");
  if (r->cfg.projection != SYMROM_DMD_DEIM)
    return fail(SYMROM_EINVAL, "rom_set_parameters: only DMD-DEIM uses the parameters");
  side_wait(r);
  return set_parameters(*r, eta, dim);
}

extern "C" symrom_status rom_dmd_state(symrom_rom* r, int32_t* S, int32_t* pstar, int32_t* rank,
                                       double* lam, double* e0, double* eh) {
  if (!r) return fail(SYMROM_EINVAL, "rom_dmd_state: null handle");
  if (!r->ready || r->cfg.projection != SYMROM_DMD_DEIM)
    return fail(SYMROM_ESTATE, "rom_dmd_state: not a DMD-DEIM handle");
  side_wait(r);
  hipStream_t s = r->s;
  if (pstar) *pstar = r->psub;
  if (S) HIPCHK(hipMemcpyAsync(S, r->sub, r->psub * sizeof(int), hipMemcpyDeviceToHost, s));
  int rk = 0;
  HIPCHK(hipMemcpyAsync(&rk, r->dmd.rdev, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // (the rank of the last DMD, at most the window width p* T <= 64)
  if (rk < 0 || rk > 64) return fail(SYMROM_EDEVICE, "rom_dmd_state: corrupt DMD rank");
  if (rank) *rank = rk;
  if (lam && rk > 0)
    HIPCHK(hipMemcpyAsync(lam, r->dmd.lam, (size_t)rk * sizeof(cplx), hipMemcpyDeviceToHost, s));
  const size_t tb = (size_t)r->p * r->Nx * sizeof(double);
  if (e0) HIPCHK(hipMemcpyAsync(e0, r->e0, tb, hipMemcpyDeviceToDevice, s));
  if (eh) HIPCHK(hipMemcpyAsync(eh, r->eh, tb, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return SYMROM_OK;
}

namespace {
struct SelBufs {
  double *psi, *colpart, *eye, *bval, *dB, *dcv;
  int *bidx, *flags;
};
SelBufs carve_sel(Arena& ar, int N, int d) {
  SelBufs b;
  b.psi = ar.take<double>((size_t)N * d);
  b.colpart = ar.take<double>((size_t)psi_blocks(N) * d);
  b.eye = ar.take<double>((size_t)d * d);
  b.bval = ar.take<double>(2 * 256);
  b.dB = ar.take<double>(2 * 64 * 64);
  b.dcv = ar.take<double>(2 * 64);
  b.bidx = ar.take<int>(2 * 256);
  b.flags = ar.take<int>(4);
  return b;
}
}  // namespace

extern "C" size_t deim_select_workspace_bytes(int32_t N, int32_t d) {
  if (N < 1 || d < 1 || d > 64 || d > N) return 0;
  Arena ar(nullptr);
  carve_sel(ar, N, d);
  return ar.off + 256;
}

extern "C" symrom_status deim_select(int32_t N, int32_t d, const double* Psi, int32_t* idx,
                                     double* w, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || d < 1 || d > 64 || d > N || !Psi || !idx || !w)
    return fail(SYMROM_EINVAL, "deim_select: bad arguments");
  if (!ws || ws_bytes < deim_select_workspace_bytes(N, d))
    return fail(SYMROM_ENOMEM, "deim_select: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  Arena ar(ws);
  SelBufs b = carve_sel(ar, N, d);
  std::vector<double> eye((size_t)d * d, 0.0);
  for (int c = 0; c < d; ++c) eye[(size_t)c * d + c] = 1.0;
  HIPCHK(hipMemcpyAsync(b.eye, eye.data(), eye.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(b.flags, 0, 4 * sizeof(int), s));
  // Psi I: a copy of the basis and its per-block column sums, as the step
  // forms them from the snapshots
  const double* in[1] = {Psi};
  launch_psi_colsum(s, in, 1, d, N, b.eye, d, d, b.psi, b.colpart);
  const int nbg = 256;
  for (int k = 0; k < d; ++k) {
    const int cur = k & 1, prev = cur ^ 1;
    launch_deim_greedy(s, b.psi, N, k, idx, b.bval + prev * nbg, b.bidx + prev * nbg, nbg, nbg,
                       b.bval + cur * nbg, b.bidx + cur * nbg, b.dB + prev * 4096,
                       b.dcv + prev * 64, b.dB + cur * 4096, b.dcv + cur * 64, b.flags);
  }
  const int last = (d - 1) & 1;
  launch_deim_weights(s, b.psi, N, d, idx, b.bval + last * nbg, b.bidx + last * nbg, nbg,
                      b.dB + last * 4096, b.dcv + last * 64, b.colpart, psi_blocks(N), w, b.flags);
  LAUNCHCHK();
  int fl = 0;
  HIPCHK(hipMemcpyAsync(&fl, b.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (fl) return fail(SYMROM_ESINGULAR, "deim_select: the basis has no finite residual left");
  return SYMROM_OK;
}

extern "C" symrom_status rom_gradient(symrom_rom* r, const double* Z, double* g, double* rho,
                                      double* Phi, double* e) {
  side_wait(r);
  if (!r || !Z || !g) return fail(SYMROM_EINVAL, "rom_gradient: null argument");
  hipStream_t s = r->s;
  const int n = r->n, p = r->p;
  r->stage1_cached = false;
  launch_z_from_real(s, Z, n, p, r->Zev);
  full_gradient(*r, r->U0, r->Zev, nullptr, true);
  launch_z_to_real(s, r->gproj, n, p, g);
  size_t gb = (size_t)p * r->Nx * 8;
  if (rho) HIPCHK(hipMemcpyAsync(rho, r->b.rho, gb, hipMemcpyDeviceToDevice, s));
  if (Phi) HIPCHK(hipMemcpyAsync(Phi, r->b.phi, gb, hipMemcpyDeviceToDevice, s));
  if (e) HIPCHK(hipMemcpyAsync(e, r->b.e, gb, hipMemcpyDeviceToDevice, s));
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  return SYMROM_OK;
}

namespace {
// H(U Z) per parameter (device [p]): the electric energy of the deposit at
// X_r = Re(U~ Z~) plus |V_r|^2 / 2, V_r = Im(U~ Z~) (the arithmetic of
// rom_diagnostics, on the handle's field and gather buffers)
void hamiltonian_of(symrom_rom& r, const cplx* U, const cplx* Z, double* H) {
  hipStream_t s = r.s;
  const int N = r.N, p = r.p, n = r.n;
  launch_deposit_rom(s, U, N, n, Z, p, r.Nx, r.gdep, r.b.factor, nullptr, r.b.part, nullptr,
                     nullptr, r.cfg.deterministic);
  launch_poisson(s, r.b.part, r.gdep.nrb, p, r.Nx, r.b.qw, r.b.h, r.b.mw, nullptr, r.b.rho,
                 r.b.phi, r.b.e, r.b.energy);
  double* Vr = reinterpret_cast<double*>(r.G);
  launch_reconstruct(s, U, N, n, Z, p, nullptr, Vr);
  launch_colsumsq(s, Vr, N, p, 0.5, H, r.b.part);
  launch_vec_add(s, H, r.b.energy, p);
}

size_t split_z_offset(const symrom_rom* r) {
  return ((size_t)r->N * r->nmax * sizeof(cplx) + 255) & ~(size_t)255;
}
}  // namespace

extern "C" size_t rom_hamiltonian_split_bytes(const symrom_rom* r) {
  if (!r) return 0;
  return split_z_offset(r) + (size_t)r->nmax * r->p * sizeof(cplx);
}

extern "C" symrom_status rom_step_hamiltonian_split(symrom_rom* r, void* scratch,
                                                    size_t scratch_bytes, double* H4,
                                                    symrom_step_info* info) {
  if (!r || !scratch || !H4) return fail(SYMROM_EINVAL, "rom_step_hamiltonian_split: null pointer");
  if (!r->ready) return fail(SYMROM_ESTATE, "rom_step_hamiltonian_split: handle not initialised");
  if (scratch_bytes < rom_hamiltonian_split_bytes(r))
    return fail(SYMROM_EINVAL, "rom_step_hamiltonian_split: scratch too small");
  if (reinterpret_cast<uintptr_t>(scratch) % 256 != 0)
    return fail(SYMROM_EINVAL, "rom_step_hamiltonian_split: scratch not 256-byte aligned");
  side_wait(r);
  const bool dmd = r->cfg.projection == SYMROM_DMD_DEIM && r->win_count + 1 >= r->nslots;
  const int p = r->p;
  r->split_U = static_cast<cplx*>(scratch);
  r->split_Z = reinterpret_cast<cplx*>(static_cast<char*>(scratch) + split_z_offset(r));
  r->last.iters_total = r->last.deim_steps = r->last.stalled_total = 0;
  symrom_status st = dmd ? rom_step_dmd(*r) : rom_step_one(*r, false);
  r->split_U = r->split_Z = nullptr;
  r->last.iters_total = r->last.iters;
  r->last.deim_steps = r->last.deim_active;
  r->last.stalled_total = r->last.stalled;
  r->last.two_n = 2 * r->n;
  if (info) *info = r->last;
  if (st != SYMROM_OK) return st;
  // after the step U_{tau-1}, Z_{tau-1} are in the exchanged buffers
  r->stage1_cached = false;
  hamiltonian_of(*r, r->Uh, r->Z1, H4);
  hamiltonian_of(*r, (const cplx*)scratch, r->Z1, H4 + p);
  hamiltonian_of(*r, (const cplx*)scratch,
                 reinterpret_cast<const cplx*>(static_cast<char*>(scratch) + split_z_offset(r)),
                 H4 + 2 * p);
  hamiltonian_of(*r, r->U0, r->Z0, H4 + 3 * p);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(r->s));
  return SYMROM_OK;
}

extern "C" symrom_status rom_autotune(symrom_rom* r, int32_t* cbn, int32_t* et_lds,
                                      int32_t* nb_max, double* best_ms, double* rule_ms) {
  if (!r) return fail(SYMROM_EINVAL, "rom_autotune: null handle");
  if (!r->ready) return fail(SYMROM_ESTATE, "rom_autotune: handle not initialised");
  if (r->cfg.deterministic)
    return fail(SYMROM_ESTATE, "rom_autotune: a deterministic handle keeps the built-in shape");
  if (!fused_gradient_ok(r->n))
    return fail(SYMROM_ESTATE, "rom_autotune: no fused gather-projection at this rank");
  side_wait(r);
  hipStream_t s = r->s;
  const int N = r->N, p = r->p, Nx = r->Nx, n = r->n;
  const size_t cap = (size_t)r->nkb * 64 * 64;
  const double qm = r->cfg.q / r->cfg.m;
  // the field and the Grams of the current state (the timed launches then
  // compute its gradient)
  r->stage1_cached = false;
  set_gather_project_shape(N, p, Nx, n, nullptr);
  const GpShape rule = gather_project_shape(N, p, Nx, n, cap);
  linear_grams(*r, r->U0, r->C12t);
  full_gradient_field(*r, r->U0, r->Z0, nullptr);
  hipEvent_t ea = nullptr, eb = nullptr;
  HIPCHK(hipEventCreate(&ea));
  if (hipEventCreate(&eb) != hipSuccess) {
    (void)hipEventDestroy(ea);
    return fail(SYMROM_EDEVICE, "rom_autotune: event");
  }
  auto launch = [&]() {
    launch_gather_project(s, r->U0, N, n, r->Z0, p, Nx, r->b.factor, r->b.e, qm, nullptr, true,
                          r->gemm_part, cap, r->gproj, r->colsq, r->C12t);
  };
  // the average of three launches after one untimed one
  auto time_shape = [&](const GpShape& sh) -> double {
    set_gather_project_shape(N, p, Nx, n, &sh);
    launch();
    float ms = -1.0f;
    if (hipEventRecord(ea, s) != hipSuccess) return -1.0;
    for (int k = 0; k < 3; ++k) launch();
    if (hipEventRecord(eb, s) != hipSuccess || hipEventSynchronize(eb) != hipSuccess ||
        hipEventElapsedTime(&ms, ea, eb) != hipSuccess || hipGetLastError() != hipSuccess)
      return -1.0;
    return ms / 3.0;
  };
  GpShape best = rule;
  double t_rule = time_shape(rule), t_best = t_rule;
  bool ok = t_rule > 0.0;
  for (const GpShape& sh : gather_project_shapes(N, p, Nx, n, cap)) {
    if (!ok) break;
    if (sh.cbn == rule.cbn && sh.et_lds == rule.et_lds && sh.nb_max == rule.nb_max) continue;
    const double t = time_shape(sh);
    if (t <= 0.0) {
      ok = false;
      break;
    }
    // another shape only when clearly faster (launch-to-launch noise is a
    // per cent or two)
    if (t < 0.97 * t_best) {
      best = sh;
      t_best = t;
    }
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  if (!ok) {
    set_gather_project_shape(N, p, Nx, n, nullptr);
    return fail(SYMROM_EDEVICE, "rom_autotune: a timed launch failed");
  }
  set_gather_project_shape(N, p, Nx, n, &best);
  if (cbn) *cbn = best.cbn;
  if (et_lds) *et_lds = best.et_lds ? 1 : 0;
  if (nb_max) *nb_max = best.nb_max;
  if (best_ms) *best_ms = t_best;
  if (rule_ms) *rule_ms = t_rule;
  return SYMROM_OK;
}

extern "C" symrom_status rom_init_singular_values(symrom_rom* r, double* sig, int32_t cap,
                                                  int32_t* m) {
  if (!r || !m || cap < 0 || (cap > 0 && !sig))
    return fail(SYMROM_EINVAL, "rom_init_singular_values: bad arguments");
  const int ns = (int)r->init_sig.size();
  for (int j = 0; j < std::min(ns, (int)cap); ++j) sig[j] = r->init_sig[j];
  *m = ns;
  return SYMROM_OK;
}

extern "C" symrom_status rom_diagnostics(symrom_rom* r, double* E, double* H) {
  side_wait(r);
  if (!r) return fail(SYMROM_EINVAL, "rom_diagnostics: null handle");
  r->stage1_cached = false;
  hipStream_t s = r->s;
  const int N = r->N, p = r->p, n = r->n;
  launch_deposit_rom(s, r->U0, N, n, r->Z0, p, r->Nx, r->gdep, r->b.factor, nullptr, r->b.part,
                     nullptr, nullptr, r->cfg.deterministic);
  launch_poisson(s, r->b.part, r->gdep.nrb, p, r->Nx, r->b.qw, r->b.h, r->b.mw, nullptr, r->b.rho,
                 r->b.phi, r->b.e, r->b.energy);
  if (E) HIPCHK(hipMemcpyAsync(E, r->b.energy, p * 8, hipMemcpyDeviceToDevice, s));
  if (H) {
    // velocities V_r = Im(U~ Z~) into the real view of the gather buffer
    double* Vr = reinterpret_cast<double*>(r->G);
    launch_reconstruct(s, r->U0, N, n, r->Z0, p, nullptr, Vr);
    launch_colsumsq(s, Vr, N, p, 0.5, H, r->b.part);
    launch_vec_add(s, H, r->b.energy, p);
  }
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  return SYMROM_OK;
}

extern "C" void rom_destroy(symrom_rom* r) {
  if (!r) return;
  side_wait(r);
  if (r->ev_fork) (void)hipEventDestroy(r->ev_fork);
  if (r->ev_sp0) (void)hipEventDestroy(r->ev_sp0);
  if (r->ev_sp1) (void)hipEventDestroy(r->ev_sp1);
  if (r->ev_join) (void)hipEventDestroy(r->ev_join);
  if (r->ev_read) (void)hipEventDestroy(r->ev_read);
  if (r->ev_join3) (void)hipEventDestroy(r->ev_join3);
  if (r->s3) {
    (void)hipStreamSynchronize(r->s3);
    (void)hipStreamDestroy(r->s3);
  }
  if (r->s2) (void)hipStreamDestroy(r->s2);
  if (r->hstat) (void)hipHostFree(r->hstat);
  delete r;
}
