// fg_noalloc.hip -- the query search for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc): fg_search_noalloc runs the kernels of fg_search with
// their scratch in a fixed array the library owns on each GPU.
//
// `scratch` below is a device global.  In host code its name is only a
// host-side stand-in; the device address of each GPU's copy is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is ever handed to kernels or fills.
#include <mutex>
#include <string>

#include "fg_internal.h"

namespace fg {
namespace {

constexpr size_t kScratchBytes = 64ull << 20;  // per GPU, held until the process ends
constexpr int kNoAllocSpillCap = 2048;         // ids listed for clearing a search's bitset
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// This device's copy of `scratch` (looked up on the device's first call).
fg_status scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(std::string("HIP error: ") + hipGetErrorString(e)), FG_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return set_error("device index beyond the no-allocation table"), FG_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)), FG_EHIP;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return FG_OK;
}

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t ctl, sgoff, sgids, deg, scan, bits, slist, total;
  int64_t words;
};

// Regions in the order of SearchScratch; `grid` bitsets and spill lists.
Layout layout(int64_t n, uint32_t R, int64_t grid) {
  Layout l{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += up256(bytes);
    return at;
  };
  const uint64_t un = (uint64_t)n;
  l.words = (n + 31) / 32;
  l.ctl = take(4096);
  l.sgoff = take((un + 1) * 8);
  l.sgids = take(((uint64_t)R * un + 2 * un + 1) * 4);
  l.deg = take(un * 4);
  l.scan = take(scan_scratch_bytes(n + 1));
  l.bits = take((size_t)grid * l.words * 4);
  l.slist = take((size_t)grid * kNoAllocSpillCap * 4);
  l.total = o;
  return l;
}

}  // namespace
}  // namespace fg

using namespace fg;

extern "C" {

size_t fg_search_noalloc_scratch_bytes(void) { return kScratchBytes; }

fg_status fg_search_noalloc(const fg_data* data, const fg_graph* graph, const void* queries_dev, int64_t nq,
                            uint32_t k, uint32_t L, uint32_t* out_ids_dev, void* out_dists_dev,
                            uint32_t* out_evals_dev, void* stream) {
  Shape s;
  fg_status r = check_search(data, graph, queries_dev, nq, k, L, out_ids_dev, out_dists_dev, &s);
  if (r) return r;
  // As many resident searches as fit the kernel and the array, at least one
  // per compute unit; below that the input is too large for this entry point.
  const int cus = num_cus_host();
  int grid = beam_grid(s, (int)L, true, 4096);
  if (grid <= 0) return set_error("no search kernel for this row size / L"), FG_EUNSUPPORTED;
  const Layout fixed = layout(s.n, graph->R, 0);
  const size_t per_slot = (size_t)fixed.words * 4 + (size_t)kNoAllocSpillCap * 4;
  const int64_t fit = fixed.total + 512 < kScratchBytes ? (int64_t)((kScratchBytes - fixed.total - 512) / per_slot) : 0;
  if (fit < cus) {
    char msg[256];
    snprintf(msg, sizeof msg,
             "fg_search_noalloc: n = %lld with R = %u needs %zu + %d x %zu bytes, beyond its %zu-byte scratch "
             "(use fg_search with a workspace)",
             (long long)s.n, graph->R, fixed.total, cus, per_slot, kScratchBytes);
    return set_error(msg), FG_EINVAL;
  }
  if (grid > fit) grid = (int)(fit / cus * cus);
  const Layout l = layout(s.n, graph->R, grid);
  if (l.total > kScratchBytes) return set_error("fg_search_noalloc: scratch layout overflow"), FG_EINVAL;
  if (nq == 0) return FG_OK;
  void* base = nullptr;
  r = scratch_ptr(&base);
  if (r) return r;
  char* b = static_cast<char*>(base);
  SearchScratch w{};
  w.ctl = b + l.ctl;
  w.sgoff = reinterpret_cast<uint64_t*>(b + l.sgoff);
  w.sgids = reinterpret_cast<uint32_t*>(b + l.sgids);
  w.deg = reinterpret_cast<uint32_t*>(b + l.deg);
  w.scan = b + l.scan;
  w.bits = reinterpret_cast<uint32_t*>(b + l.bits);
  w.spill_words = l.words;
  w.slist = reinterpret_cast<uint32_t*>(b + l.slist);
  w.spill_cap = kNoAllocSpillCap;
  return search_run(s, graph, queries_dev, nq, k, L, out_ids_dev, out_dists_dev, out_evals_dev, w, grid,
                    static_cast<hipStream_t>(stream));
}

}  // extern "C"
