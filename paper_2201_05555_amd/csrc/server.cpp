// Serving loop for ensembles of parameter queries: requests (a family, its
// parameters eta, shared uniforms and a step count) arrive at any time;
// each is admitted when a slot is free and its reduced model fits the device
// memory pool the caller handed over (its exact workspace plus its uniforms,
// from rom_workspace_bytes), and is then run on a stream of its own by a
// worker thread: device-side loading and the truncated complex SVD
// (rom_init_family), the steps (rom_step), the diagnostics and the requested
// rows of R = U Z.  U and Z stay resident in the request's workspace for all
// its steps; requests never share an ensemble (U depends on all of its
// parameters), so their work overlaps on the device without mixing.  The
// pool is the only device memory used: admission is by its free space.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/symrom.h"

namespace {
double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit sub-allocator over [0, size) with 256-byte granules.
struct Pool {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  size_t used = 0, peak = 0;
  void init(void* b, size_t s) {
    base = static_cast<char*>(b);
    size = s & ~size_t(255);
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t o2 = it->first + n;
        free_.erase(it);
        if (rest) free_[o2] = rest;
        used += n;
        peak = std::max(peak, used);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~size_t(255);
    used -= n;
    auto it = free_.emplace(off, n).first;
    // merge with the next and the previous free ranges
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Request {
  int64_t id = 0;
  symrom_config cfg{};
  int32_t family = 0;
  std::vector<double> eta, ux, uv;
  int32_t nsteps = 0;
  std::vector<int32_t> rows;
  // results
  std::vector<double> E, H, Xr, Vr;
  symrom_request_info info{};  // read and written under the server's mutex
  size_t off = 0, bytes = 0;
  std::string error;
  // written by the worker while it runs the request, published under the
  // mutex when it finishes
  symrom_status result = SYMROM_OK;
  int32_t two_n = 0;
};

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// device bytes a request occupies while it runs: its workspace, the two
// uniform streams, eta and the row list, the diagnostics and the sampled rows
size_t request_bytes(const symrom_config& c, int32_t nrows) {
  const size_t ws = rom_workspace_bytes(&c);
  if (!ws) return 0;
  return align256(ws) + 2 * align256((size_t)c.N * 8) + align256((size_t)c.p * 32) +
         align256((size_t)std::max(nrows, 1) * 4) + 2 * align256((size_t)c.p * 8) +
         2 * align256((size_t)std::max(nrows, 1) * c.p * 8);
}
}  // namespace

struct symrom_server {
  int device = 0;
  int slots = 0;
  Pool pool;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> pending, ready;
  std::map<int64_t, std::shared_ptr<Request>> all;
  int running = 0;
  int64_t next_id = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  double t0 = 0.0;

  // admit pending requests in arrival order while a slot and pool space allow
  // (a request that does not fit does not block the smaller ones behind it)
  void admit_locked() {
    for (auto it = pending.begin(); it != pending.end() && running < slots;) {
      auto& r = *it;
      size_t off = 0;
      if (pool.alloc(r->bytes, &off)) {
        r->off = off;
        r->info.status = 2;
        ++running;
        ready.push_back(r);
        it = pending.erase(it);
        cv_work.notify_one();
      } else {
        ++it;
      }
    }
  }

  void run(Request& r, hipStream_t s) {
    char* base = pool.base + r.off;
    size_t o = 0;
    auto take = [&](size_t n) {
      char* p = base + o;
      o += align256(n);
      return p;
    };
    const int N = r.cfg.N, p = r.cfg.p;
    const int nr = (int)r.rows.size();
    const size_t ws_bytes = rom_workspace_bytes(&r.cfg);
    void* ws = take(ws_bytes);
    double* ux = reinterpret_cast<double*>(take((size_t)N * 8));
    double* uv = reinterpret_cast<double*>(take((size_t)N * 8));
    take((size_t)p * 32);
    int32_t* rows = reinterpret_cast<int32_t*>(take((size_t)std::max(nr, 1) * 4));
    double* E = reinterpret_cast<double*>(take((size_t)p * 8));
    double* H = reinterpret_cast<double*>(take((size_t)p * 8));
    double* X = reinterpret_cast<double*>(take((size_t)std::max(nr, 1) * p * 8));
    double* V = reinterpret_cast<double*>(take((size_t)std::max(nr, 1) * p * 8));
    auto fail = [&](const char* what) { r.error = std::string(what) + ": " + symrom_last_error(); };
    if (hipMemcpyAsync(ux, r.ux.data(), (size_t)N * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(uv, r.uv.data(), (size_t)N * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        (nr && hipMemcpyAsync(rows, r.rows.data(), (size_t)nr * 4, hipMemcpyHostToDevice, s) !=
                   hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess) {
      r.result = SYMROM_EDEVICE;
      r.error = "upload";
      return;
    }
    symrom_rom* h = nullptr;
    symrom_status st =
        rom_init_family(&r.cfg, r.family, r.eta.data(), ux, uv, ws, ws_bytes, s, &h);
    if (st != SYMROM_OK) {
      r.result = st;
      fail("rom_init_family");
      return;
    }
    symrom_step_info si{};
    st = rom_step(h, r.nsteps, &si);
    if (st == SYMROM_OK) st = rom_diagnostics(h, E, H);
    if (st == SYMROM_OK && nr) st = rom_reconstruct_rows(h, rows, nr, X, V);
    int32_t two_n = 0;
    if (st == SYMROM_OK) st = rom_get_state(h, nullptr, nullptr, &two_n, nullptr);
    if (st == SYMROM_OK) {
      r.E.resize(p);
      r.H.resize(p);
      r.Xr.resize((size_t)nr * p);
      r.Vr.resize((size_t)nr * p);
      if (hipMemcpyAsync(r.E.data(), E, (size_t)p * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipMemcpyAsync(r.H.data(), H, (size_t)p * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
          (nr && (hipMemcpyAsync(r.Xr.data(), X, (size_t)nr * p * 8, hipMemcpyDeviceToHost, s) !=
                      hipSuccess ||
                  hipMemcpyAsync(r.Vr.data(), V, (size_t)nr * p * 8, hipMemcpyDeviceToHost, s) !=
                      hipSuccess)) ||
          hipStreamSynchronize(s) != hipSuccess)
        st = SYMROM_EDEVICE;
    } else {
      fail("step");
    }
    r.two_n = two_n;
    rom_destroy(h);
    r.result = st;
  }

  void worker() {
    if (hipSetDevice(device) != hipSuccess) return;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
      std::shared_ptr<Request> r;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || !ready.empty(); });
        if (ready.empty()) break;  // stop requested and nothing left
        r = ready.front();
        ready.pop_front();
      }
      const double ts = now_s() - t0;
      run(*r, s);
      (void)hipStreamSynchronize(s);
      const double tf = now_s() - t0;
      {
        std::lock_guard<std::mutex> lk(mu);
        r->info.t_start = ts;
        r->info.t_finish = tf;
        r->info.two_n = r->two_n;
        r->info.steps_done = (r->result == SYMROM_OK) ? r->nsteps : -1;
        r->info.status = r->result;
        pool.release(r->off, r->bytes);
        --running;
        // the request's host copies of its inputs are no longer needed
        r->ux.clear();
        r->ux.shrink_to_fit();
        r->uv.clear();
        r->uv.shrink_to_fit();
        admit_locked();
      }
      cv_done.notify_all();
    }
    (void)hipStreamDestroy(s);
  }
};

extern "C" size_t srv_request_bytes(const symrom_config* cfg, int32_t nrows) {
  if (!cfg || nrows < 0) return 0;
  return request_bytes(*cfg, nrows);
}

extern "C" symrom_status srv_create(int32_t slots, void* pool, size_t pool_bytes,
                                    symrom_server** out) {
  if (slots < 1 || slots > 64 || !pool || pool_bytes < 4096 || !out) return SYMROM_EINVAL;
  symrom_server* sv = new symrom_server();
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return SYMROM_EDEVICE;
  }
  sv->slots = slots;
  sv->pool.init(pool, pool_bytes);
  sv->t0 = now_s();
  for (int i = 0; i < slots; ++i) sv->workers.emplace_back([sv] { sv->worker(); });
  *out = sv;
  return SYMROM_OK;
}

extern "C" symrom_status srv_submit(symrom_server* sv, const symrom_config* cfg, int32_t family,
                                    const double* eta, const double* ux, const double* uv,
                                    int32_t nsteps, int32_t nrows, const int32_t* rows,
                                    int64_t* id) {
  if (!sv || !cfg || !eta || !ux || !uv || nsteps < 0 || nrows < 0 || (nrows && !rows) ||
      (family != 0 && family != 1))
    return SYMROM_EINVAL;
  const size_t bytes = request_bytes(*cfg, nrows);
  if (!bytes) return SYMROM_EINVAL;
  if (bytes > sv->pool.size) return SYMROM_ENOMEM;  // could never be admitted
  auto r = std::make_shared<Request>();
  r->cfg = *cfg;
  r->family = family;
  r->eta.assign(eta, eta + 4 * (size_t)cfg->p);
  r->ux.assign(ux, ux + cfg->N);
  r->uv.assign(uv, uv + cfg->N);
  r->nsteps = nsteps;
  r->rows.assign(rows, rows + nrows);
  r->bytes = bytes;
  r->info.status = 1;
  r->info.pp_steps = (double)cfg->N * cfg->p * nsteps;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    r->id = sv->next_id++;
    r->info.t_arrival = now_s() - sv->t0;
    sv->all[r->id] = r;
    sv->pending.push_back(r);
    sv->admit_locked();
  }
  if (id) *id = r->id;
  return SYMROM_OK;
}

extern "C" symrom_status srv_info(symrom_server* sv, int64_t id, symrom_request_info* info) {
  if (!sv || !info) return SYMROM_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return SYMROM_EINVAL;
  *info = it->second->info;
  return SYMROM_OK;
}

extern "C" symrom_status srv_wait(symrom_server* sv, int64_t id) {
  if (!sv) return SYMROM_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return SYMROM_EINVAL;
  auto r = it->second;
  sv->cv_done.wait(lk, [&] { return r->info.status <= 0; });
  return r->info.status;
}

extern "C" symrom_status srv_drain(symrom_server* sv, double* peak_pool_bytes) {
  if (!sv) return SYMROM_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv_done.wait(lk, [&] { return sv->pending.empty() && sv->ready.empty() && sv->running == 0; });
  if (peak_pool_bytes) *peak_pool_bytes = (double)sv->pool.peak;
  return SYMROM_OK;
}

extern "C" symrom_status srv_result(symrom_server* sv, int64_t id, double* E, double* H,
                                    double* X, double* V) {
  if (!sv) return SYMROM_EINVAL;
  std::shared_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return SYMROM_EINVAL;
    r = it->second;
    if (r->info.status > 0) return SYMROM_ESTATE;  // not finished
  }
  if (r->info.status != SYMROM_OK) return r->info.status;
  if (E) std::memcpy(E, r->E.data(), r->E.size() * 8);
  if (H) std::memcpy(H, r->H.data(), r->H.size() * 8);
  if (X) std::memcpy(X, r->Xr.data(), r->Xr.size() * 8);
  if (V) std::memcpy(V, r->Vr.data(), r->Vr.size() * 8);
  return SYMROM_OK;
}

extern "C" void srv_destroy(symrom_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->pending.clear();
  }
  sv->cv_work.notify_all();
  for (auto& t : sv->workers) t.join();
  delete sv;
}
