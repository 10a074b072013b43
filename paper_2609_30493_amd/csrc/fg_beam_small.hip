// fg_beam_small.hip -- plain harvest kernels with a small on-chip visited
// table (512 or 1024 slots, ef_h <= 128), for every row shape.
//
// A search whose visits outgrow its table continues in the device bitset,
// and an expanded set longer than half the table is sorted and pruned in
// device memory, so the table size never changes the graph; a smaller table
// leaves LDS for more resident searches per compute unit, which hide more of
// the dependent gathers' latency when most searches spill anyway.
#include "fg_internal.h"

namespace fg {

namespace {

template <int DK, int L, int NCH>
void* pick_ef_small(int ef, int hslots) {
  if (ef <= 64)
    return hslots == 512 ? reinterpret_cast<void*>(&k_beam<DK, L, NCH, 64, 512, false>)
                         : reinterpret_cast<void*>(&k_beam<DK, L, NCH, 64, 1024, false>);
  if (ef <= 128)
    return hslots == 512 ? reinterpret_cast<void*>(&k_beam<DK, L, NCH, 128, 512, false>)
                         : reinterpret_cast<void*>(&k_beam<DK, L, NCH, 128, 1024, false>);
  return nullptr;
}

}  // namespace

void* pick_small(int dk, int Q, int ef, int hslots) {
  if (hslots != 512 && hslots != 1024) return nullptr;
  if (dk == U8L2) {
    if (Q <= 8) return pick_ef_small<U8L2, 8, 1>(ef, hslots);
    if (Q <= 16) return pick_ef_small<U8L2, 16, 1>(ef, hslots);
    return nullptr;
  }
#define FG_F32_ROWS(DKV)                                       \
  if (Q <= 8) return pick_ef_small<DKV, 8, 1>(ef, hslots);     \
  if (Q <= 16) return pick_ef_small<DKV, 16, 1>(ef, hslots);   \
  if (Q <= 32) return pick_ef_small<DKV, 16, 2>(ef, hslots);   \
  if (Q <= 64) return pick_ef_small<DKV, 16, 4>(ef, hslots);   \
  if (Q <= 256) return pick_ef_small<DKV, 16, 16>(ef, hslots); \
  return nullptr;
  if (dk == F32L2) { FG_F32_ROWS(F32L2) }
  if (dk == F32COS) { FG_F32_ROWS(F32COS) }
#undef FG_F32_ROWS
  return nullptr;
}

}  // namespace fg

#ifdef FG_PROFILE
FG_PROF_READER(fg_prof_read_small)
#endif
