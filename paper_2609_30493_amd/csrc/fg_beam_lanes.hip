// fg_beam_lanes.hip -- harvest kernels with another number of lanes per row.
//
// The declared summation order gives the same bits for any L in {1, 2, 4,
// 8, 16} lanes sharing a row (the 16 partials are spread over the group's
// lanes, combined in the same tree), so the lanes per row is a pure tuning
// knob: fewer lanes per row hold more chunks each and put more rows in
// flight per wave.  The alternatives instantiated here (plain harvest only;
// the default shapes are in fg_beam.hip):
//   rows of at most  8 chunks: 4 lanes x 2 chunks   (default 8 x 1)
//   rows of  9..16 chunks:     8 lanes x 2 chunks   (default 16 x 1)
//   rows of 17..32 chunks:     8 lanes x 4 chunks   (default 16 x 2)
#include "fg_internal.h"

namespace fg {

namespace {

template <int DK, int L, int NCH>
void* pick_ef_lanes(int ef, int hslots) {
  const bool big = hslots == 4096;
  if (ef <= 64)
    return big ? reinterpret_cast<void*>(&k_beam<DK, L, NCH, 64, 4096, false>)
               : reinterpret_cast<void*>(&k_beam<DK, L, NCH, 64, 2048, false>);
  if (ef <= 128)
    return big ? reinterpret_cast<void*>(&k_beam<DK, L, NCH, 128, 4096, false>)
               : reinterpret_cast<void*>(&k_beam<DK, L, NCH, 128, 2048, false>);
  if (ef <= 256) return reinterpret_cast<void*>(&k_beam<DK, L, NCH, 256, 4096, false>);
  return nullptr;
}

}  // namespace

void* pick_lanes(int dk, int Q, int ef, int hslots, int lanes) {
  int L = 0, nch = 0;
  if (!lanes_variant(dk, Q, lanes, &L, &nch)) return nullptr;
#define FG_LANES(DKV)                                                  \
  if (L == 4 && nch == 2) return pick_ef_lanes<DKV, 4, 2>(ef, hslots); \
  if (L == 8 && nch == 2) return pick_ef_lanes<DKV, 8, 2>(ef, hslots); \
  if (DKV != U8L2 && L == 8 && nch == 4) return pick_ef_lanes<DKV, 8, 4>(ef, hslots);
  if (dk == U8L2) { FG_LANES(U8L2) }
  if (dk == F32L2) { FG_LANES(F32L2) }
  if (dk == F32COS) { FG_LANES(F32COS) }
#undef FG_LANES
  return nullptr;
}

bool lanes_variant(int dk, int Q, int lanes, int* L, int* nch) {
  *L = 0;
  *nch = 0;
  if (lanes == 4 && Q <= 8) {
    *L = 4;
    *nch = 2;
  } else if (lanes == 8 && Q > 8 && Q <= 16) {
    *L = 8;
    *nch = 2;
  } else if (lanes == 8 && dk != U8L2 && Q > 16 && Q <= 32) {
    *L = 8;
    *nch = 4;
  }
  return *L != 0;
}

}  // namespace fg
