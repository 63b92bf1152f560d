// C ABI of the LOVE library: argument validation, cache allocation, build
// orchestration, query dispatch and the optional per-kernel event timer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace love;

// ----------------------------------------------------------------------------
// Kernel timing
// ----------------------------------------------------------------------------
namespace {
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
struct ProfState {
  std::mutex mu;
  bool on = false;
  std::vector<ProfRec> pending;
  std::vector<std::pair<std::string, hipEvent_t>> open;  // begin events by name (stack)
  std::map<std::string, std::pair<int64_t, double>> acc;
  std::vector<hipEvent_t> pool;
  std::vector<std::string> select;   // empty: time every scope
};
ProfState& prof() {
  static ProfState* p = new ProfState();
  return *p;
}
hipEvent_t take_event(ProfState& p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}
void drain(ProfState& p) {
  for (auto& r : p.pending) {
    hipEventSynchronize(r.b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, r.a, r.b);
    auto& slot = p.acc[r.name];
    slot.first += 1;
    slot.second += ms;
    p.pool.push_back(r.a);
    p.pool.push_back(r.b);
  }
  p.pending.clear();
}
}  // namespace

namespace love {
bool prof_on() { return prof().on; }
void prof_begin(const char* name, hipStream_t s) {
  ProfState& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  if (!p.select.empty() && std::find(p.select.begin(), p.select.end(), name) == p.select.end()) return;
  hipEvent_t e = take_event(p);
  hipEventRecord(e, s);
  p.open.emplace_back(name, e);
}
bool prof_kernel_events(const char* name, hipEvent_t* start, hipEvent_t* stop) {
  ProfState& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  if (!p.select.empty() && std::find(p.select.begin(), p.select.end(), name) == p.select.end())
    return false;
  if (p.pending.size() > 4096) drain(p);   // before the new pair: its kernel is not queued yet
  *start = take_event(p);
  *stop = take_event(p);
  p.pending.push_back({name, *start, *stop});
  return true;
}
void prof_end(const char* name, hipStream_t s) {
  ProfState& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  for (size_t i = p.open.size(); i-- > 0;) {
    if (p.open[i].first == name) {
      hipEvent_t b = take_event(p);
      hipEventRecord(b, s);
      p.pending.push_back({name, p.open[i].second, b});
      p.open.erase(p.open.begin() + i);
      break;
    }
  }
  if (p.pending.size() > 4096) drain(p);
}

void* mem_alloc(const MemSource& m, size_t bytes, hipStream_t s) {
  if (m.user) return m.a.alloc(bytes, (void*)s, m.a.ctx);
  void* p = nullptr;
  return hipMallocAsync(&p, bytes, s) == hipSuccess ? p : nullptr;
}

void mem_free(const MemSource& m, void* p, hipStream_t s) {
  if (!p) return;
  if (m.user) m.a.free(p, (void*)s, m.a.ctx);
  else (void)hipFreeAsync(p, s);
}

namespace {
const MemSource& pool_source() {
  static const MemSource pool{};
  return pool;
}
thread_local const MemSource* t_mem = nullptr;
}  // namespace

const MemSource& cur_mem() { return t_mem ? *t_mem : pool_source(); }

MemScope::MemScope(const MemSource& m) : prev_(t_mem), mine_(m) { t_mem = &mine_; }
MemScope::~MemScope() { t_mem = prev_; }

// Cache memory comes from the build call's source on the cache's stream (the
// device's stream-ordered pool keeps freed memory for the next build, with no
// device-wide synchronisation) and goes back to it in love_cache_free.
bool dev_reserve(love_cache* c, size_t bytes) {
  void* p = mem_alloc(c->mem, bytes, c->stream);
  if (!p) return false;
  c->allocs.push_back(p);
  c->block = (char*)p;
  c->block_size = bytes;
  c->block_used = 0;
  return true;
}

void* dev_alloc(love_cache* c, size_t bytes) {
  bytes = dev_round(bytes);
  c->bytes += bytes;
  if (c->block && c->block_used + bytes <= c->block_size) {
    void* p = c->block + c->block_used;
    c->block_used += bytes;
    return p;
  }
  void* p = mem_alloc(c->mem, bytes, c->stream);
  if (!p) return nullptr;
  c->allocs.push_back(p);
  return p;
}
}  // namespace love

// ----------------------------------------------------------------------------
// Validation
// ----------------------------------------------------------------------------
static love_status validate(const love_config* cfg) {
  if (!cfg) return LOVE_EINVAL;
  if (cfg->d < 1 || cfg->d > LOVE_MAX_DIM) return LOVE_EINVAL;
  const bool add = cfg->flags & LOVE_FLAG_ADDITIVE;
  int64_t mt = add ? 0 : 1, ct = add ? 0 : 1;
  for (int e = 0; e < cfg->d; ++e) {
    if (cfg->m[e] < 4) return LOVE_EINVAL;
    if (!(cfg->hi[e] > cfg->lo[e]) || !std::isfinite(cfg->lo[e]) || !std::isfinite(cfg->hi[e]))
      return LOVE_EINVAL;
    if (!(cfg->lengthscale[e] > 0) || !std::isfinite(cfg->lengthscale[e])) return LOVE_EINVAL;
    if (add) {
      if (cfg->m[e] > (1 << 24)) return LOVE_EINVAL;
      mt += cfg->m[e];
      ct += cfg->m[e] - 3;
    } else {
      mt *= cfg->m[e];
      ct *= cfg->m[e] - 3;
    }
    if (mt > (int64_t(1) << 31) || ct > (int64_t(1) << 30)) return LOVE_EINVAL;
  }
  if (!(cfg->outputscale > 0) || !std::isfinite(cfg->outputscale)) return LOVE_EINVAL;
  if (!(cfg->noise > 0) || !std::isfinite(cfg->noise)) return LOVE_EINVAL;
  if (cfg->kernel != LOVE_RBF && cfg->kernel != LOVE_MATERN52) return LOVE_EINVAL;
  if (cfg->k < 1 || cfg->k > LOVE_MAX_K) return LOVE_EINVAL;
  if (cfg->k_sample < 0 || cfg->k_sample > LOVE_MAX_K) return LOVE_EINVAL;
  if (cfg->precision < LOVE_P_FP64 || cfg->precision > LOVE_P_FP32_BF16SPLIT) return LOVE_EINVAL;
  if (cfg->toeplitz < LOVE_TOEPLITZ_AUTO || cfg->toeplitz > LOVE_TOEPLITZ_FFT) return LOVE_EINVAL;
  if (cfg->cg_tol < 0 || !std::isfinite(cfg->cg_tol)) return LOVE_EINVAL;
  if (!std::isfinite(cfg->restart_tol)) return LOVE_EINVAL;
  if (cfg->restart_tol > 0 && (cfg->flags & LOVE_FLAG_HYPER)) return LOVE_EUNSUPPORTED;
  if (cfg->restart_tol > 0) {
    const int rmax = cfg->restart_max > 0 ? cfg->restart_max : 1;
    if (cfg->restart_k < 1 || (int64_t)cfg->k + (int64_t)rmax * cfg->restart_k > LOVE_MAX_K)
      return LOVE_EINVAL;
    if (cfg->restart_groups > (1 << 16)) return LOVE_EINVAL;
  }
  return LOVE_OK;
}

static int kround(int k) { return k <= 64 ? 64 : 128; }

static love_status init_cache(love_cache* c, const love_config* cfg, int64_t n, hipStream_t s) {
  c->cfg = *cfg;
  c->mem = cur_mem();
  c->fp64 = cfg->precision == LOVE_P_FP64;
  c->d = cfg->d;
  c->n = n;
  c->stream = s;
  (void)hipGetDevice(&c->device);
  c->add = (cfg->flags & LOVE_FLAG_ADDITIVE) != 0;
  int64_t m = c->add ? 0 : 1, ct = c->add ? 0 : 1;
  for (int e = 0; e < 4; ++e) {
    if (e < c->d) {
      c->mdim[e] = cfg->m[e];
      c->lo[e] = cfg->lo[e];
      c->hi[e] = cfg->hi[e];
      c->invh[e] = (double)(cfg->m[e] - 3) / (cfg->hi[e] - cfg->lo[e]);
      if (c->add) {
        c->aoff[e] = m;
        c->acoff[e] = ct;
        m += cfg->m[e];
        ct += cfg->m[e] - 3;
      } else {
        m *= cfg->m[e];
        ct *= cfg->m[e] - 3;
      }
    } else {
      c->mdim[e] = 1;
      c->lo[e] = c->hi[e] = 0.0;
      c->invh[e] = 0.0;
    }
  }
  c->m = m;
  c->ctot = ct;
  c->ldq = cdiv(n, RB) * RB;
  // k: Lanczos vectors the buffers hold (the first run's k1 plus the
  // restarts' steps); the first run takes k1
  c->k1 = (int)std::min<int64_t>(cfg->k, n);
  if (cfg->restart_tol > 0) {
    c->restart_max = cfg->restart_max > 0 ? cfg->restart_max : 1;
    c->restart_groups = cfg->restart_groups > 0 ? cfg->restart_groups : 8;
    c->restart_k = cfg->restart_k;
  }
  c->k = (int)std::min<int64_t>((int64_t)c->k1 + (int64_t)c->restart_max * c->restart_k, n);
  c->kpad = kround(c->k);
  c->ks = (int)std::min<int64_t>(cfg->k_sample, m);
  c->kspad = c->ks > 0 ? kround(c->ks) : 0;
  c->tol_lanczos = c->fp64 ? 1e-12 : 1e-8;
  const size_t es = c->fp64 ? 8 : 4;
  const bool split = cfg->precision == LOVE_P_FP32_BF16SPLIT;
  {
    // everything the cache keeps, in one block: the buffers below, the
    // Toeplitz coefficient columns and first-four table, the Toeplitz scratch
    const size_t nperm = (size_t)n * (c->add ? c->d : 1);
    size_t want = dev_round(es * (size_t)n * c->d) + dev_round(es * (size_t)n) +
                  dev_round(4 * nperm) + dev_round(4 * (size_t)(ct + 1)) +
                  dev_round(2 * sizeof(Ctl) + 4 * sizeof(unsigned)) + dev_round(sizeof(double)) +
                  2 * dev_round(sizeof(double) * LOVE_MAX_K) +
                  dev_round((split ? 2 : es) * (size_t)m * c->kpad) +
                  (split ? dev_round(2 * (size_t)m * c->kpad) : 0) + dev_round(es * (size_t)m) +
                  (c->ks > 0 ? dev_round(sizeof(float) * (size_t)m * c->kspad) : 0) +
                  ((cfg->flags & LOVE_FLAG_HYPER) ? dev_round(es * (size_t)m * c->kpad) : 0) +
                  2 * dev_round(es * (size_t)n) + 2 * dev_round(es * (size_t)m) +
                  dev_round(sizeof(double) * 16) +
                  dev_round(sizeof(double) * (size_t)toeplitz_scratch_elems(c));
    for (int e = 0; e < c->d; ++e)
      want += dev_round(8 * (size_t)cfg->m[e]) + dev_round(4 * (size_t)cfg->m[e]);
    if (!dev_reserve(c, want)) return LOVE_ENOMEM;
  }
  c->x = dev_alloc(c, es * (size_t)n * c->d);
  c->y = dev_alloc(c, es * (size_t)n);
  c->perm = (int32_t*)dev_alloc(c, 4 * (size_t)n * (c->add ? c->d : 1));
  c->cell_start = (int32_t*)dev_alloc(c, 4 * (size_t)(ct + 1));
  // the two control blocks and the status words are contiguous (one clear)
  c->ctl = (Ctl*)dev_alloc(c, 2 * sizeof(Ctl) + 4 * sizeof(unsigned));
  c->ctl_s = c->ctl ? c->ctl + 1 : nullptr;
  c->status = c->ctl ? (unsigned*)(c->ctl + 2) : nullptr;
  c->ortho = (double*)dev_alloc(c, sizeof(double));
  c->alpha = (double*)dev_alloc(c, sizeof(double) * LOVE_MAX_K);
  c->beta = (double*)dev_alloc(c, sizeof(double) * LOVE_MAX_K);
  c->rt = dev_alloc(c, (split ? 2 : es) * (size_t)m * c->kpad);
  if (split) c->rt_lo = dev_alloc(c, 2 * (size_t)m * c->kpad);
  c->a = dev_alloc(c, es * (size_t)m);
  if (c->ks > 0) c->S = (float*)dev_alloc(c, sizeof(float) * (size_t)m * c->kspad);
  if (cfg->flags & LOVE_FLAG_HYPER) c->B = dev_alloc(c, es * (size_t)m * c->kpad);
  c->v1 = dev_alloc(c, es * (size_t)n);
  c->v2 = dev_alloc(c, es * (size_t)n);
  c->g1 = dev_alloc(c, es * (size_t)m);
  c->g2 = dev_alloc(c, es * (size_t)m);
  c->tscr = nullptr;  // allocated after the Toeplitz plan
  if (!c->x || !c->y || !c->perm || !c->cell_start || !c->ctl || !c->ctl_s || !c->status || !c->ortho ||
      !c->alpha || !c->beta || !c->rt || (split && !c->rt_lo) || !c->a || (c->ks > 0 && !c->S) ||
      !c->v1 || !c->v2 || !c->g1 || !c->g2 || ((cfg->flags & LOVE_FLAG_HYPER) && !c->B))
    return LOVE_ENOMEM;
  LOVE_HIP_TRY(hipMemsetAsync(c->ctl, 0, 2 * sizeof(Ctl) + 4 * sizeof(unsigned), s));
  LOVE_HIP_TRY(hipMemsetAsync(c->a, 0, es * (size_t)m, s));
  return LOVE_OK;
}

// Stream-ordered release on the cache's stream: work queued there before the
// call completes first; the host does not wait.
static void destroy(love_cache* c) {
  if (!c) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != c->device) (void)hipSetDevice(c->device);
  for (void* p : c->allocs) mem_free(c->mem, p, c->stream);
  if (cur != c->device) (void)hipSetDevice(cur);
  delete c;
}

static love_status finish_status(love_cache* c) {
  // ctl, ctl_s and the status words are contiguous: one copy
  struct {
    Ctl h, hs;
    unsigned st[4];
  } b;
  static_assert(sizeof(b) == 2 * sizeof(Ctl) + 4 * sizeof(unsigned), "control block layout");
  LOVE_HIP_TRY(hipMemcpyAsync(&b, c->ctl, sizeof(b), hipMemcpyDeviceToHost, c->stream));
  LOVE_HIP_TRY(hipStreamSynchronize(c->stream));
  const Ctl& h = b.h;
  c->keff_h = h.k_eff;
  c->kseff_h = c->ks > 0 ? b.hs.k_chol : 0;
  c->keff_known = 1;
  const unsigned all = h.status | b.st[0];
  if (all & SF_DOMAIN) return LOVE_EDOMAIN;
  if (all & SF_NONFINITE) return LOVE_ENONFINITE;
  if (h.k_eff < 1) return LOVE_ENOTPD;
  return LOVE_OK;
}

// Once per device: the stream-ordered allocator keeps freed memory in its pool
// instead of returning it to the driver at every synchronisation, so the
// per-build scratch (hipMallocAsync / hipFreeAsync) is reused without driver
// calls.
static void device_setup() {
  static std::mutex mu;
  static std::map<int, bool> done;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(mu);
  if (done[dev]) return;
  done[dev] = true;
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool) {
    uint64_t keep = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
}

// One non-blocking side stream per device for the sampler chain (default priority).
static hipStream_t side_stream() {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  streams[dev] = st;
  return st;
}

// One non-blocking stream per device for the grid-space mean solve, which runs
// beside the Lanczos (default priority).
hipStream_t love::mean_stream() {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  streams[dev] = st;
  return st;
}

// Build a batch of caches (same d and precision) with one launch per phase.
template <typename T>
static love_status build_batch(const std::vector<love_cache*>& cs, const void* const* xs,
                               const void* const* ys, hipStream_t s) {
  const int G = (int)cs.size();
  std::vector<const T*> xv(G), yv(G);
  for (int g = 0; g < G; ++g) {
    xv[g] = (const T*)xs[g];
    yv[g] = (const T*)ys[g];
  }
  love_status st = setup_sort<T>(cs, xv, yv, s);
  if (st != LOVE_OK) return st;
  bool any_s = false;
  for (auto* c : cs) {
    st = toeplitz_plan(c);
    if (st != LOVE_OK) return st;
    c->tscr = dev_alloc(c, sizeof(double) * (size_t)toeplitz_scratch_elems(c));
    if (!c->tscr) return LOVE_ENOMEM;
    any_s = any_s || c->ks > 0;
  }
  return build_batch_lanczos<T>(cs, s, any_s ? side_stream() : nullptr);
}

template <typename T>
static love_status apply_khat_t(const love_cache* c, const T* v, T* out, hipStream_t s) {
  love_cache* cm = const_cast<love_cache*>(c);
  std::vector<love_cache*> one{cm};
  JobArena A;
  ScatterJob<T> S{};
  S.g = make_grid<T>(c);
  S.x = (const T*)c->x;
  S.cell_start = c->cell_start;
  S.v = (const T*)c->v1;
  S.out = (T*)c->g1;
  void* cellp = nullptr;
  const size_t cb = scatter_scratch_bytes(c, sizeof(T));
  if (cb && !(cellp = ws_alloc(cb, s))) return LOVE_ENOMEM;
  S.cellp = (T*)cellp;
  GatherJob<T> Ga{};
  Ga.g = S.g;
  Ga.x = S.x;
  Ga.n = c->n;
  Ga.kg = (const T*)c->g2;
  Ga.vsig = (const T*)c->v1;
  Ga.sigma2 = (T)c->cfg.noise;
  Ga.out = (T*)c->v2;
  const size_t os = A.add(std::vector<ScatterJob<T>>{S});
  const size_t og = A.add(std::vector<GatherJob<T>>{Ga});
  ToepRun<T> run;
  toep_prepare<T>(A, run, one, {(const T*)c->g1}, {0}, {(T*)c->g2}, {0}, {(T*)c->tscr}, {nullptr});
  love_status st = A.upload(s);
  if (st != LOVE_OK) {
    ws_free(cellp, s);
    return st;
  }
  // rows of an additive cache stay in caller order (perm holds the axes' cell lists)
  if (c->add) LOVE_HIP_TRY(hipMemcpyAsync(c->v1, v, sizeof(T) * c->n, hipMemcpyDeviceToDevice, s));
  else launch_permute<T>(v, (T*)c->v1, c->perm, c->n, 0, s);
  launch_scatter<T>(tab1(cdiv(c->m, 4)), A.at<ScatterJob<T>>(os), c->d, 0, 0, s,
                    scatter_kinds(one));
  toep_run<T>(A, run, 0, 0, s);
  launch_gather<T>(tab1(cdiv(c->n, 256)), A.at<GatherJob<T>>(og), c->d, 0, s);
  if (c->add) LOVE_HIP_TRY(hipMemcpyAsync(out, c->v2, sizeof(T) * c->n, hipMemcpyDeviceToDevice, s));
  else launch_permute<T>((const T*)c->v2, out, c->perm, c->n, 1, s);
  A.release(s);
  ws_free(cellp, s);
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}

template <typename T>
static love_status apply_kuu_t(const love_cache* c, const T* g, T* out, hipStream_t s) {
  std::vector<love_cache*> one{const_cast<love_cache*>(c)};
  JobArena A;
  ToepRun<T> run;
  toep_prepare<T>(A, run, one, {g}, {0}, {out}, {0}, {(T*)c->tscr}, {nullptr});
  love_status st = A.upload(s);
  if (st != LOVE_OK) return st;
  toep_run<T>(A, run, 0, 0, s);
  A.release(s);
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}

extern "C" {

int32_t love_abi_version(void) { return LOVE_ABI_VERSION; }

const char* love_status_string(love_status s) {
  switch (s) {
    case LOVE_OK: return "ok";
    case LOVE_EINVAL: return "invalid argument";
    case LOVE_EDOMAIN: return "point outside the grid domain";
    case LOVE_ENOTPD: return "Lanczos tridiagonal not positive definite";
    case LOVE_ENOMEM: return "device out of memory";
    case LOVE_EHIP: return "HIP runtime error";
    case LOVE_ENONFINITE: return "non-finite value";
    case LOVE_EUNSUPPORTED: return "unsupported request";
    case LOVE_ELIMIT: return "request exceeds a fixed limit of the call";
  }
  return "unknown status";
}

// The memory source an entry point was given (NULL: the device's pool).
static bool mem_source(const love_allocator* a, MemSource* m) {
  *m = MemSource{};
  if (!a) return true;
  if (!a->alloc || !a->free) return false;
  m->a = *a;
  m->user = true;
  return true;
}

love_status love_build_cache(const love_config* cfg, const void* x, const void* y, int64_t n,
                             const love_allocator* alloc, void* stream, love_cache** out) {
  return love_build_cache_batched(1, cfg, &x, &y, &n, alloc, stream, out);
}

love_status love_build_cache_batched(int32_t G, const love_config* cfgs, const void* const* xs,
                                     const void* const* ys, const int64_t* ns,
                                     const love_allocator* alloc, void* stream,
                                     love_cache** out) {
  if (G < 1 || !cfgs || !xs || !ys || !ns || !out) return LOVE_EINVAL;
  MemSource ms;
  if (!mem_source(alloc, &ms)) return LOVE_EINVAL;
  for (int g = 0; g < G; ++g) {
    love_status st = validate(&cfgs[g]);
    if (st != LOVE_OK) return st;
    if (cfgs[g].precision != cfgs[0].precision || cfgs[g].d != cfgs[0].d) return LOVE_EINVAL;
    if (!xs[g] || !ys[g] || ns[g] < 1 || ns[g] > INT32_MAX) return LOVE_EINVAL;
    if ((cfgs[g].flags & LOVE_FLAG_NO_MEAN) != (cfgs[0].flags & LOVE_FLAG_NO_MEAN))
      return LOVE_EINVAL;
    if ((cfgs[g].flags & LOVE_FLAG_ADDITIVE) != (cfgs[0].flags & LOVE_FLAG_ADDITIVE))
      return LOVE_EINVAL;
    if (G > 1 && cfgs[g].restart_tol > 0) return LOVE_EUNSUPPORTED;   // restarts: single builds
  }
  hipStream_t s = (hipStream_t)stream;
  device_setup();
  MemScope scope(ms);
  std::vector<love_cache*> made;
  auto fail = [&](love_status st) {
    for (auto* p : made) destroy(p);
    return st;
  };
  for (int g = 0; g < G; ++g) {
    love_cache* c = new (std::nothrow) love_cache();
    if (!c) return fail(LOVE_ENOMEM);
    made.push_back(c);
    love_status st = init_cache(c, &cfgs[g], ns[g], s);
    if (st != LOVE_OK) return fail(st);
  }
  // lock-step groups of at most MAXG GPs
  for (int g0 = 0; g0 < G; g0 += MAXG) {
    const int g1 = std::min(G, g0 + MAXG);
    std::vector<love_cache*> grp(made.begin() + g0, made.begin() + g1);
    love_status st = made[0]->fp64 ? build_batch<double>(grp, xs + g0, ys + g0, s)
                                    : build_batch<float>(grp, xs + g0, ys + g0, s);
    if (st != LOVE_OK) return fail(st);
  }
  for (int g = 0; g < G; ++g) {
    love_status st = (cfgs[g].flags & LOVE_FLAG_ASYNC) ? LOVE_OK : finish_status(made[g]);
    if (st != LOVE_OK) return fail(st);
  }
  for (int g = 0; g < G; ++g) out[g] = made[g];
  return LOVE_OK;
}

love_status love_predict_mean_var(const love_cache* c, const void* xs, int64_t t, void* mean,
                                  void* var, void* stream) {
  return love_predict_mean_var_batched(1, &c, &xs, &t, &mean, &var, stream);
}

love_status love_predict_mean_var_batched(int32_t G, const love_cache* const* caches,
                                          const void* const* xs, const int64_t* ts,
                                          void* const* means, void* const* vars, void* stream) {
  if (G < 1 || !caches || !xs || !ts || !vars) return LOVE_EINVAL;
  for (int g = 0; g < G; ++g) {
    if (!caches[g] || ts[g] < 0 || (ts[g] > 0 && (!xs[g] || !vars[g]))) return LOVE_EINVAL;
    if (caches[g]->fp64 != caches[0]->fp64 || caches[g]->d != caches[0]->d ||
        caches[g]->cfg.precision != caches[0]->cfg.precision)
      return LOVE_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<const love_cache*> cs(caches, caches + G);
  std::vector<int64_t> tv(ts, ts + G);
  if (caches[0]->fp64) {
    std::vector<const double*> x(G);
    std::vector<double*> mu(G), va(G);
    for (int g = 0; g < G; ++g) {
      x[g] = (const double*)xs[g];
      mu[g] = means ? (double*)means[g] : nullptr;
      va[g] = (double*)vars[g];
    }
    return predict_batch<double>(cs, x, tv, mu, va, s);
  }
  std::vector<const float*> x(G);
  std::vector<float*> mu(G), va(G);
  for (int g = 0; g < G; ++g) {
    x[g] = (const float*)xs[g];
    mu[g] = means ? (float*)means[g] : nullptr;
    va[g] = (float*)vars[g];
  }
  return predict_batch<float>(cs, x, tv, mu, va, s);
}

love_status love_predict_covar_pairs(const love_cache* c, const void* xa, const void* xb,
                                     int64_t t, void* cov, void* stream) {
  if (!c || t < 0 || (t > 0 && (!xa || !xb || !cov))) return LOVE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  MemScope scope(c->mem);
  if (c->fp64) return covar_pairs<double>(c, (const double*)xa, (const double*)xb, t, (double*)cov, s);
  return covar_pairs<float>(c, (const float*)xa, (const float*)xb, t, (float*)cov, s);
}

love_status love_predict_covar_block(const love_cache* c, const void* xa, int64_t ta,
                                     const void* xb, int64_t tb, void* cov,
                                     const love_allocator* alloc, void* stream) {
  if (!c || ta < 0 || tb < 0 || (ta > 0 && tb > 0 && (!xa || !xb || !cov))) return LOVE_EINVAL;
  MemSource ms;
  if (!mem_source(alloc, &ms)) return LOVE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  MemScope scope(alloc ? ms : c->mem);
  if (c->fp64)
    return covar_block<double>(c, (const double*)xa, ta, (const double*)xb, tb, (double*)cov, s);
  return covar_block<float>(c, (const float*)xa, ta, (const float*)xb, tb, (float*)cov, s);
}

love_status love_sample_posterior(const love_cache* c, const void* xs, int64_t t, const float* z,
                                  int64_t ns, void* out, void* stream) {
  if (!c || t < 0 || ns < 0 || (t > 0 && ns > 0 && (!xs || !z || !out))) return LOVE_EINVAL;
  if (c->ks <= 0) return LOVE_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  MemScope scope(c->mem);
  if (c->fp64) return sample<double>(c, (const double*)xs, t, z, ns, (double*)out, s);
  return sample<float>(c, (const float*)xs, t, z, ns, (float*)out, s);
}

love_status love_sample_posterior_noalloc(const love_cache* c, const void* xs, int64_t t,
                                          const float* z, int64_t ns, void* out, void* stream) {
  if (!c || t < 0 || ns < 0 || (t > 0 && ns > 0 && (!xs || !z || !out))) return LOVE_EINVAL;
  if (c->ks <= 0) return LOVE_EUNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LOVE_EHIP;
  if (dev != c->device) return LOVE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (c->fp64) return sample_noalloc<double>(c, (const double*)xs, t, z, ns, (double*)out, s);
  return sample_noalloc<float>(c, (const float*)xs, t, z, ns, (float*)out, s);
}

love_status love_predict_backward(const love_cache* c, const void* xs, int64_t t,
                                  const void* g_mean, const void* g_var, void* g_xs, float* g_rt,
                                  void* stream) {
  if (!c || t < 0 || (t > 0 && (!xs || !g_xs))) return LOVE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  MemScope scope(c->mem);
  if (c->fp64)
    return backward<double>(c, (const double*)xs, t, (const double*)g_mean, (const double*)g_var,
                            (double*)g_xs, g_rt, s);
  return backward<float>(c, (const float*)xs, t, (const float*)g_mean, (const float*)g_var,
                         (float*)g_xs, g_rt, s);
}

love_status love_predict_var_hyper_grad(const love_cache* c, const void* xs, int64_t t,
                                        const void* g_var, double* grad, void* stream) {
  if (!c || t < 0 || !grad || (t > 0 && (!xs || !g_var))) return LOVE_EINVAL;
  if (!c->B) return LOVE_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  MemScope scope(c->mem);
  ProfScope ps("hyper_grad", s);
  if (c->fp64)
    return hyper_grad<double>(c, (const double*)xs, t, (const double*)g_var, grad, s);
  return hyper_grad<float>(c, (const float*)xs, t, (const float*)g_var, grad, s);
}

love_status love_apply_khat(const love_cache* c, const void* v, void* out, void* stream) {
  if (!c || !v || !out) return LOVE_EINVAL;
  if (c->n == 0) return LOVE_EUNSUPPORTED;   // imported cache: no training rows
  hipStream_t s = (hipStream_t)stream;
  MemScope scope(c->mem);
  ProfScope ps("apply_khat", s);
  if (c->fp64) return apply_khat_t<double>(c, (const double*)v, (double*)out, s);
  return apply_khat_t<float>(c, (const float*)v, (float*)out, s);
}

love_status love_apply_kuu(const love_cache* c, const void* g, void* out, void* stream) {
  if (!c || !g || !out) return LOVE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  MemScope scope(c->mem);
  if (c->fp64) return apply_kuu_t<double>(c, (const double*)g, (double*)out, s);
  return apply_kuu_t<float>(c, (const float*)g, (float*)out, s);
}

love_status love_cache_info(const love_cache* c, love_cache_info_t* info) {
  if (!c || !info) return LOVE_EINVAL;
  Ctl h, hs;
  unsigned st[4];
  LOVE_HIP_TRY(hipMemcpyAsync(&h, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  LOVE_HIP_TRY(hipMemcpyAsync(&hs, c->ctl_s, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  LOVE_HIP_TRY(hipMemcpyAsync(st, c->status, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  double bl = 0.0, orth = 0.0;
  if (h.k_eff > 0)
    LOVE_HIP_TRY(hipMemcpyAsync(&bl, c->beta + h.k_eff - 1, sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
  LOVE_HIP_TRY(hipMemcpyAsync(&orth, c->ortho, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LOVE_HIP_TRY(hipStreamSynchronize(c->stream));
  std::memset(info, 0, sizeof(*info));
  info->k_eff = h.k_eff;
  info->k_eff_sample = c->ks > 0 ? hs.k_chol : 0;
  info->cg_iters = h.cg_iters;
  info->d = c->d;
  info->n = c->n;
  info->m = c->m;
  info->beta_last = bl;
  info->ortho_loss = (c->cfg.flags & (LOVE_FLAG_NO_MEAN | LOVE_FLAG_PLAIN_CG)) ? NAN : orth;
  info->status_flags = h.status | hs.status | st[0];
  for (int e = 0; e < c->d; ++e) {
    info->toeplitz_mode[e] = (uint32_t)c->toep.ax[e].mode;
    info->fft_len[e] = (uint32_t)(c->toep.ax[e].mode == 2 ? c->toep.ax[e].fft_n : 0);
  }
  info->bytes = c->bytes;
  info->restarts = c->restarts;
  info->solve_residual = c->solve_residual;
  return LOVE_OK;
}

love_status love_cache_keff(const love_cache* c, int32_t* k_eff, int32_t* k_eff_sample) {
  if (!c || !k_eff || !k_eff_sample) return LOVE_EINVAL;
  if (!c->keff_known) {
    love_cache_info_t info;
    love_status st = love_cache_info(c, &info);
    if (st != LOVE_OK) return st;
    *k_eff = info.k_eff;
    *k_eff_sample = info.k_eff_sample;
    return LOVE_OK;
  }
  *k_eff = c->keff_h;
  *k_eff_sample = c->kseff_h;
  return LOVE_OK;
}

love_status love_cache_export(const love_cache* c, const love_export* e, void* stream) {
  if (!c || !e) return LOVE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Ctl h, hs;
  LOVE_HIP_TRY(hipMemcpyAsync(&h, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  LOVE_HIP_TRY(hipMemcpyAsync(&hs, c->ctl_s, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  LOVE_HIP_TRY(hipStreamSynchronize(s));
  const int k = h.k_eff;
  const size_t es = c->fp64 ? 8 : 4;
  if (e->alpha) LOVE_HIP_TRY(hipMemcpyAsync(e->alpha, c->alpha, sizeof(double) * k, hipMemcpyDeviceToDevice, s));
  if (e->beta) LOVE_HIP_TRY(hipMemcpyAsync(e->beta, c->beta, sizeof(double) * k, hipMemcpyDeviceToDevice, s));
  if (e->a) LOVE_HIP_TRY(hipMemcpyAsync(e->a, c->a, es * c->m, hipMemcpyDeviceToDevice, s));
  if (e->rt) {
    love_status st = rt_export_f32(c, e->rt, k, s);
    if (st != LOVE_OK) return st;
  }
  if (e->rt64) {
    if (!c->fp64) return LOVE_EINVAL;
    LOVE_HIP_TRY(hipMemcpy2DAsync(e->rt64, sizeof(double) * k, c->rt, sizeof(double) * c->kpad,
                                  sizeof(double) * k, c->m, hipMemcpyDeviceToDevice, s));
  }
  if (e->s && c->ks > 0 && hs.k_chol > 0)
    LOVE_HIP_TRY(hipMemcpy2DAsync(e->s, sizeof(float) * hs.k_chol, c->S, sizeof(float) * c->kspad,
                                  sizeof(float) * hs.k_chol, c->m, hipMemcpyDeviceToDevice, s));
  return LOVE_OK;
}

love_status love_cache_import(const love_config* cfg, const love_import* im,
                              const love_allocator* alloc, void* stream, love_cache** out) {
  if (!cfg || !im || !out) return LOVE_EINVAL;
  *out = nullptr;
  MemSource ms;
  if (!mem_source(alloc, &ms)) return LOVE_EINVAL;
  love_status st = validate(cfg);
  if (st != LOVE_OK) return st;
  if (im->k_eff < 1 || im->k_eff > LOVE_MAX_K || im->k_eff_sample < 0 ||
      im->k_eff_sample > LOVE_MAX_K)
    return LOVE_EINVAL;
  const bool fp64 = cfg->precision == LOVE_P_FP64;
  if (fp64 ? !im->rt64 : !im->rt) return LOVE_EINVAL;
  if ((im->k_eff_sample > 0) != (im->s != nullptr)) return LOVE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  device_setup();
  MemScope scope(ms);
  love_config cf = *cfg;
  cf.k = im->k_eff;
  cf.k_sample = im->k_eff_sample;
  love_cache* c = new (std::nothrow) love_cache();
  if (!c) return LOVE_ENOMEM;
  // the row-sized buffers are sized for k_eff rows (unused: no training data)
  st = init_cache(c, &cf, im->k_eff, s);
  if (st == LOVE_OK) st = toeplitz_plan(c);
  if (st == LOVE_OK) {
    c->tscr = dev_alloc(c, sizeof(double) * (size_t)toeplitz_scratch_elems(c));
    if (!c->tscr) st = LOVE_ENOMEM;
  }
  if (st == LOVE_OK) st = rt_import(c, im->rt, im->rt64, im->k_eff, im->k_eff_sample, s);
  const size_t es = c->fp64 ? 8 : 4;
  auto copy = [&](void* dst, const void* src, size_t bytes) {
    if (st == LOVE_OK && hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
      st = LOVE_EHIP;
  };
  auto clear = [&](void* dst, size_t bytes) {
    if (st == LOVE_OK && hipMemsetAsync(dst, 0, bytes, s) != hipSuccess) st = LOVE_EHIP;
  };
  clear(c->alpha, sizeof(double) * LOVE_MAX_K);
  clear(c->beta, sizeof(double) * LOVE_MAX_K);
  if (im->alpha) copy(c->alpha, im->alpha, sizeof(double) * im->k_eff);
  if (im->beta) copy(c->beta, im->beta, sizeof(double) * im->k_eff);
  if (im->a) copy(c->a, im->a, es * (size_t)c->m);
  if (c->ks > 0) {
    clear(c->S, sizeof(float) * (size_t)c->m * c->kspad);
    if (st == LOVE_OK &&
        hipMemcpy2DAsync(c->S, sizeof(float) * c->kspad, im->s, sizeof(float) * im->k_eff_sample,
                         sizeof(float) * im->k_eff_sample, c->m, hipMemcpyDeviceToDevice,
                         s) != hipSuccess)
      st = LOVE_EHIP;
  }
  if (st != LOVE_OK) {
    destroy(c);
    return st;
  }
  c->n = 0;   // no training rows: love_apply_khat is unavailable
  c->keff_h = im->k_eff;
  c->kseff_h = im->k_eff_sample;
  c->keff_known = 1;
  *out = c;
  return LOVE_OK;
}

void love_cache_free(love_cache* c) { destroy(c); }

love_status love_profile_enable(int32_t enable) {
  ProfState& p = prof();
  hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(p.mu);
  drain(p);
  if (enable) p.acc.clear();
  p.on = enable != 0;
  return LOVE_OK;
}

love_status love_profile_select(const char* names) {
  ProfState& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.select.clear();
  if (!names) return LOVE_OK;
  std::string all(names);
  size_t start = 0;
  while (start < all.size()) {
    size_t comma = all.find(',', start);
    if (comma == std::string::npos) comma = all.size();
    if (comma > start) p.select.push_back(all.substr(start, comma - start));
    start = comma + 1;
  }
  return LOVE_OK;
}

love_status love_profile_read(const char* names, int64_t* calls, double* ms) {
  if (!names || !calls || !ms) return LOVE_EINVAL;
  ProfState& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  drain(p);
  std::string all(names);
  size_t i = 0, start = 0;
  while (start <= all.size()) {
    size_t comma = all.find(',', start);
    if (comma == std::string::npos) comma = all.size();
    std::string nm = all.substr(start, comma - start);
    auto it = p.acc.find(nm);
    calls[i] = it == p.acc.end() ? 0 : it->second.first;
    ms[i] = it == p.acc.end() ? 0.0 : it->second.second;
    ++i;
    start = comma + 1;
    if (comma == all.size()) break;
  }
  return LOVE_OK;
}

}  // extern "C"
