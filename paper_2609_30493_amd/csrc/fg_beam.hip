// fg_beam.hip -- instantiation and dispatch of the beam kernels.
//
// A kernel is chosen by (distance kind, lanes per row L, chunks per lane NCH,
// beam bound EFMAX): L lanes share one row so that a group reads 16*L
// contiguous bytes per step; L*NCH must cover the row's 16-byte chunks.
#include "fg_internal.h"

namespace fg {

namespace {

template <int DK, int L, int NCH, int EFMAX, bool SEARCH>
void* kernel_ptr(int hslots) {
  if (hslots == 2048) return reinterpret_cast<void*>(&k_beam<DK, L, NCH, EFMAX, 2048, SEARCH>);
  return reinterpret_cast<void*>(&k_beam<DK, L, NCH, EFMAX, 4096, SEARCH>);
}

template <int DK, int L, int NCH, bool SEARCH>
void* pick_ef(int ef, int hslots) {
  if constexpr (SEARCH) {
    if (ef <= 128) return kernel_ptr<DK, L, NCH, 128, SEARCH>(4096);
    if (ef <= 512) return kernel_ptr<DK, L, NCH, 512, SEARCH>(4096);
  } else {
    if (ef <= 64) return kernel_ptr<DK, L, NCH, 64, SEARCH>(hslots);
    if (ef <= 128) return kernel_ptr<DK, L, NCH, 128, SEARCH>(hslots);
    if (ef <= 256) return kernel_ptr<DK, L, NCH, 256, SEARCH>(4096);
  }
  return nullptr;
}

template <bool SEARCH>
void* pick(int dk, int Q, int ef, int hslots) {
  if (dk == U8L2) {
    if (Q <= 8) return pick_ef<U8L2, 8, 1, SEARCH>(ef, hslots);
    if (Q <= 16) return pick_ef<U8L2, 16, 1, SEARCH>(ef, hslots);
    return nullptr;
  }
#define FG_F32_ROWS(DKV)                                                 \
  if (Q <= 8) return pick_ef<DKV, 8, 1, SEARCH>(ef, hslots);             \
  if (Q <= 16) return pick_ef<DKV, 16, 1, SEARCH>(ef, hslots);           \
  if (Q <= 32) return pick_ef<DKV, 16, 2, SEARCH>(ef, hslots);           \
  if (Q <= 64) return pick_ef<DKV, 16, 4, SEARCH>(ef, hslots);           \
  if (Q <= 256) return pick_ef<DKV, 16, 16, SEARCH>(ef, hslots);         \
  return nullptr;
  if (dk == F32L2) { FG_F32_ROWS(F32L2) }
  if (dk == F32COS) { FG_F32_ROWS(F32COS) }
#undef FG_F32_ROWS
  return nullptr;
}

int num_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 256;
  }
  return cus;
}

}  // namespace

int num_cus_host() { return num_cus(); }

int beam_chunks_per_lane(const Shape& s, int lanes) {
  int L = 0, nch = 0;
  if (lanes && lanes_variant(s.dk, s.Q, lanes, &L, &nch)) return nch;
  if (s.Q <= 16) return 1;
  if (s.Q <= 32) return 2;
  if (s.Q <= 64) return 4;
  return 16;
}

// Slots of the on-chip visited table actually used for this launch: the
// search kernels and ef > 128 always use 4096; otherwise `hslots` (512,
// 1024, 2048 or 4096) as requested.
int beam_table_slots(int ef, bool search, int hslots, int nch) {
  (void)nch;
  if (search || ef > 128) return 4096;
  if (hslots == 512 || hslots == 1024 || hslots == 2048) return hslots;
  return 4096;
}

static void* pick_kernel(const Shape& s, int ef, bool search, int hslots, int screen, int lanes) {
  if (screen == kBeamLog) return search ? nullptr : pick_log(s.dk, s.Q, ef);
  if (lanes && !search && screen == SCR_NONE) {
    if (void* k = pick_lanes(s.dk, s.Q, ef, hslots, lanes)) return k;
  }
  if (!search && screen == SCR_NONE && (hslots == 512 || hslots == 1024)) return pick_small(s.dk, s.Q, ef, hslots);
  if (screen == SCR_BF16) return search ? nullptr : pick_screen_bf16(s.dk, s.Q, ef, hslots);
  if (screen == SCR_FP8) return search ? nullptr : pick_screen_fp8(s.dk, s.Q, ef, hslots);
  if (screen == SCR_INT8) return search ? nullptr : pick_screen_int8(s.dk, s.Q, ef, hslots);
  return search ? pick<true>(s.dk, s.Q, ef, hslots) : pick<false>(s.dk, s.Q, ef, hslots);
}

int beam_grid(const Shape& s, int ef, bool search, int hslots, int screen, int waves_per_cu, int lanes) {
  void* k = pick_kernel(s, ef, search, hslots, screen, lanes);
  if (!k) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k), 64, 0) !=
          hipSuccess ||
      per_cu <= 0)
    per_cu = 4;
  if (waves_per_cu > 0 && waves_per_cu < per_cu) per_cu = waves_per_cu;
  int g = per_cu * num_cus();
  return g < kMaxWaveSlots ? g : kMaxWaveSlots;
}

hipError_t launch_beam(const Shape& s, BeamArgs& a, bool search, int grid, int hslots, hipStream_t st,
                       int screen, int lanes) {
  void* k = pick_kernel(s, a.ef, search, hslots, screen, lanes);
  if (!k) return hipErrorInvalidValue;
  void* args[] = {&a};
  return hipLaunchKernel(reinterpret_cast<const void*>(k), dim3(grid), dim3(64), args, 0, st);
}

}  // namespace fg

#ifdef FG_PROFILE
// Profiling builds only: read and clear this unit's phase cycle counters.
FG_PROF_READER(fg_prof_read)
#endif
