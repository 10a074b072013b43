// fg_beam_log.hip -- the harvest kernels with the visit log (Sec. 5.5's
// lockstep-density measurement): the same search, prune and counters, plus
// the ids each logged point's search visits.  One table size (4096 slots,
// which never changes the graph) keeps the instantiations few.
#include "fg_internal.h"

namespace fg {

namespace {

template <int DK, int L, int NCH>
void* pick_ef_log(int ef) {
  if (ef <= 64) return reinterpret_cast<void*>(&k_beam<DK, L, NCH, 64, 4096, false, SCR_NONE, true>);
  if (ef <= 128) return reinterpret_cast<void*>(&k_beam<DK, L, NCH, 128, 4096, false, SCR_NONE, true>);
  if (ef <= 256) return reinterpret_cast<void*>(&k_beam<DK, L, NCH, 256, 4096, false, SCR_NONE, true>);
  return nullptr;
}

}  // namespace

void* pick_log(int dk, int Q, int ef) {
  if (dk == U8L2) {
    if (Q <= 8) return pick_ef_log<U8L2, 8, 1>(ef);
    if (Q <= 16) return pick_ef_log<U8L2, 16, 1>(ef);
    return nullptr;
  }
#define FG_F32_ROWS(DKV)                              \
  if (Q <= 8) return pick_ef_log<DKV, 8, 1>(ef);      \
  if (Q <= 16) return pick_ef_log<DKV, 16, 1>(ef);    \
  if (Q <= 32) return pick_ef_log<DKV, 16, 2>(ef);    \
  if (Q <= 64) return pick_ef_log<DKV, 16, 4>(ef);    \
  if (Q <= 256) return pick_ef_log<DKV, 16, 16>(ef);  \
  return nullptr;
  if (dk == F32L2) { FG_F32_ROWS(F32L2) }
  if (dk == F32COS) { FG_F32_ROWS(F32COS) }
#undef FG_F32_ROWS
  return nullptr;
}

}  // namespace fg
