// Event-bracketed launch records for fosb_profile_* (see include/fosb.h), and
// the auxiliary context of the concurrent pipeline.
#include <functional>

#include "common.h"

namespace fosb {

ProfScope::ProfScope(Context& c, int cls, double flops, double bytes)
    : ctx(c.prof_root ? *c.prof_root : c), stream(c.stream) {
  if (!ctx.prof_on) return;
  std::lock_guard<std::mutex> lock(ctx.prof_mu);
  const int ev = (int)(2 * ctx.recs.size());
  while ((int)ctx.ev_pool.size() < ev + 2) {
    hipEvent_t e;
    FOSB_HIP(hipEventCreate(&e));
    ctx.ev_pool.push_back(e);
  }
  FOSB_HIP(hipEventRecord(ctx.ev_pool[ev], stream));
  ctx.recs.push_back(ProfRec{cls, ev, flops, bytes});
  idx = ev;
}

ProfScope::~ProfScope() {
  if (idx < 0) return;
  std::lock_guard<std::mutex> lock(ctx.prof_mu);
  (void)hipEventRecord(ctx.ev_pool[idx + 1], stream);
}

// ------------------------------------------------------------------ caching pool
static size_t pool_round(size_t n) {
  const size_t small = (size_t)1 << 20, big = (size_t)2 << 20;
  return n < small ? (n + 4095) / 4096 * 4096 : (n + big - 1) / big * big;
}

void* Pool::get(size_t n, size_t& cap) {
  const size_t want = pool_round(n);
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = free_blocks.lower_bound(want);
    // reuse the smallest cached block that fits, unless it is more than twice the request
    if (it != free_blocks.end() && it->first <= 2 * want) {
      void* p = it->second;
      cap = it->first;
      cached_bytes -= cap;
      live_bytes += cap;
      free_blocks.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    trim();  // give the cached blocks back and try once more
    e = hipMalloc(&p, want);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? FOSB_E_OOM : FOSB_E_DEVICE, "device allocation of %zu bytes failed: %s", want,
         hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lock(mu);
  ++n_device_allocs;
  live_bytes += want;
  cap = want;
  return p;
}

void Pool::put(void* p, size_t cap) {
  std::lock_guard<std::mutex> lock(mu);
  free_blocks.emplace(cap, p);
  cached_bytes += cap;
  live_bytes -= cap;
}

void Pool::trim() {
  std::multimap<size_t, void*> blocks;
  {
    std::lock_guard<std::mutex> lock(mu);
    blocks.swap(free_blocks);
    cached_bytes = 0;
  }
  for (auto& b : blocks) (void)hipFree(b.second);
}

Pool::~Pool() { trim(); }

std::shared_ptr<Pool>& thread_pool() {
  static thread_local std::shared_ptr<Pool> tl;
  return tl;
}

void bind_pool(Context& ctx) { thread_pool() = ctx.pool; }

bool& thread_no_alloc() {
  static thread_local bool flag = false;
  return flag;
}

Context::Context() {
  for (DevBuf& b : scratch) b.home = pool;
  for (DevBuf& b : ss) b.home = pool;
  for (DevBuf* b : {&solve_tmp, &counters, &small, &norms, &splitk, &tune_out}) b->home = pool;
}

static void for_each_context(Context& c, const std::function<void(Context&)>& f) {
  f(c);
  if (c.aux) for_each_context(*c.aux, f);
  if (c.la) for_each_context(*c.la, f);
  for (auto& w : c.workers) for_each_context(*w, f);
}

void pool_totals(Context& ctx, int64_t& n_allocs, int64_t& cached, int64_t& live) {
  n_allocs = cached = live = 0;
  for_each_context(ctx, [&](Context& c) {
    std::lock_guard<std::mutex> lock(c.pool->mu);
    n_allocs += c.pool->n_device_allocs;
    cached += (int64_t)c.pool->cached_bytes;
    live += (int64_t)c.pool->live_bytes;
  });
}

void pool_trim(Context& ctx) {
  for_each_context(ctx, [&](Context& c) { c.pool->trim(); });
}

// ------------------------------------------------------------------ child contexts
static std::unique_ptr<Context> child_context(Context& parent) {
  std::unique_ptr<Context> a(new Context());
  a->device = parent.device;
  a->n_cu = parent.n_cu;
  a->max_lds = parent.max_lds;
  a->prof_root = parent.prof_root ? parent.prof_root : &parent;
  FOSB_HIP(hipSetDevice(parent.device));
  FOSB_HIP(hipStreamCreateWithFlags(&a->stream, hipStreamNonBlocking));  // default priority
  a->owns_stream = true;
  return a;
}

Context& Context::aux_context() {
  if (!aux) aux = child_context(*this);
  return *aux;
}

Context& Context::la_context() {
  if (!la) la = child_context(*this);
  return *la;
}

Context& Context::worker_context(size_t i) {
  while (workers.size() <= i) workers.push_back(child_context(*this));
  return *workers[i];
}

Context::~Context() {
  workers.clear();
  if (aux) aux.reset();
  if (la) la.reset();
  for (hipEvent_t e : lu_ev)
    if (e) (void)hipEventDestroy(e);
  if (owns_stream && stream) {
    (void)hipStreamSynchronize(stream);
    (void)hipStreamDestroy(stream);
  }
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : tune_ev)
    if (e) (void)hipEventDestroy(e);
}

}  // namespace fosb
