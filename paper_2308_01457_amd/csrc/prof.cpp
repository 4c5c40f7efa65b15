// Event-bracketed launch records for fosb_profile_* (see include/fosb.h).
#include "common.h"

namespace fosb {

ProfScope::ProfScope(Context& c, int cls, double flops, double bytes) : ctx(c) {
  if (!ctx.prof_on) return;
  const int ev = (int)(2 * ctx.recs.size());
  while ((int)ctx.ev_pool.size() < ev + 2) {
    hipEvent_t e;
    FOSB_HIP(hipEventCreate(&e));
    ctx.ev_pool.push_back(e);
  }
  FOSB_HIP(hipEventRecord(ctx.ev_pool[ev], ctx.stream));
  ctx.recs.push_back(ProfRec{cls, ev, flops, bytes});
  idx = ev;
}

ProfScope::~ProfScope() {
  if (idx >= 0) (void)hipEventRecord(ctx.ev_pool[idx + 1], ctx.stream);
}

Context::~Context() {
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
}

}  // namespace fosb
