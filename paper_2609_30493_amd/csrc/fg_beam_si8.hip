// fg_beam_si8.hip -- the screened harvest kernels with the int8 narrow copy
// (float32 rows of more than 16 chunks, L = 16 lanes per row).
#include "fg_internal.h"

namespace fg {

namespace {

template <int DK, int NCH, int EFMAX>
void* kp(int hslots) {
  if constexpr (EFMAX <= 128) {
    if (hslots == 2048) return reinterpret_cast<void*>(&k_beam<DK, 16, NCH, EFMAX, 2048, false, SCR_INT8>);
    if constexpr (NCH <= 4)
      if (hslots == 1024) return reinterpret_cast<void*>(&k_beam<DK, 16, NCH, EFMAX, 1024, false, SCR_INT8>);
  }
  return reinterpret_cast<void*>(&k_beam<DK, 16, NCH, EFMAX, 4096, false, SCR_INT8>);
}

template <int DK, int NCH>
void* pick_ef(int ef, int hslots) {
  if (ef <= 64) return kp<DK, NCH, 64>(hslots);
  if (ef <= 128) return kp<DK, NCH, 128>(hslots);
  if (ef <= 256) return kp<DK, NCH, 256>(4096);
  return nullptr;
}

template <int DK>
void* pick_q(int Q, int ef, int hslots) {
  if (Q <= 16) return nullptr;
  if (Q <= 32) return pick_ef<DK, 2>(ef, hslots);
  if (Q <= 64) return pick_ef<DK, 4>(ef, hslots);
  if (Q <= 256) return pick_ef<DK, 16>(ef, hslots);
  return nullptr;
}

}  // namespace

void* pick_screen_int8(int dk, int Q, int ef, int hslots) {
  if (dk == F32L2) return pick_q<F32L2>(Q, ef, hslots);
  if (dk == F32COS) return pick_q<F32COS>(Q, ef, hslots);
  return nullptr;
}

}  // namespace fg

#ifdef FG_PROFILE
FG_PROF_READER(fg_prof_read_si8)
#endif
