// Event-bracketed launch records for fosb_profile_* (see include/fosb.h), and
// the auxiliary context of the concurrent pipeline.
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
