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

Context& Context::aux_context() {
  if (!aux) {
    std::unique_ptr<Context> a(new Context());
    a->device = device;
    a->n_cu = n_cu;
    a->max_lds = max_lds;
    a->prof_root = this;
    FOSB_HIP(hipSetDevice(device));
    FOSB_HIP(hipStreamCreateWithFlags(&a->stream, hipStreamNonBlocking));
    a->owns_stream = true;
    aux = std::move(a);
  }
  return *aux;
}

Context::~Context() {
  if (aux) aux.reset();
  if (owns_stream && stream) {
    (void)hipStreamSynchronize(stream);
    (void)hipStreamDestroy(stream);
  }
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
}

}  // namespace fosb
