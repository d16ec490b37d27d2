// hqc_capi.cpp -- the C ABI of include/hqc_gpu.h: argument validation,
// launch configuration, hipGraph cache, per-item baseline mode, keystore.
#include "hqc_gpu.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "hqc_internal.h"
#include "hqc_internal_enc.h"

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return HQC_EHIP;
}

int pid_bit(int pid) { return pid == 1 ? 1 : pid == 3 ? 2 : pid == 5 ? 4 : 0; }

// Device memory check: [p, p + bytes) must lie inside one device allocation.
// This keeps a wrong count or a host pointer from reaching a kernel.
bool in_device_allocation(const void *p, size_t bytes) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return false;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  const char *b = (const char *)base, *q = (const char *)p;
  return q >= b && (size_t)(q - b) <= size && bytes <= size - (size_t)(q - b);
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

struct Grid {
  std::mutex mu;
  std::map<std::tuple<int, int, unsigned, int>, int> cache;  // (device, op, mask, shape) -> grid
  std::map<int, int> cus;                                    // device -> compute units
};
Grid g_grid;

// The occupancy grid (CUs x resident workgroups) of a kernel on the current
// device, cached per device; *cus_out (optional) gets the CU count.
int default_grid(int op, unsigned mask, int *out, int shape = 0, int *cus_out = nullptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  std::lock_guard<std::mutex> lk(g_grid.mu);
  auto key = std::make_tuple(dev, op, mask, shape);
  auto it = g_grid.cache.find(key);
  auto ct = g_grid.cus.find(dev);
  if (it != g_grid.cache.end() && ct != g_grid.cus.end()) {
    *out = it->second;
    if (cus_out) *cus_out = ct->second;
    return HQC_OK;
  }
  int cus = 0, per_cu = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e);
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, hqc::kernel_ptr(op, mask, shape), 64,
                                                   hqc::lds_bytes_for(op, mask, shape));
  if (e != hipSuccess) return hip_fail(e);
  if (per_cu < 1) per_cu = 1;
  *out = cus * per_cu;
  g_grid.cache[key] = *out;
  g_grid.cus[dev] = cus;
  if (cus_out) *cus_out = cus;
  return HQC_OK;
}

// hipGraph cache: one instantiated graph per distinct launch.
struct GraphKey {
  int op;
  unsigned mask;
  int shape;
  int grid;
  int device;
  std::vector<unsigned char> args;
  bool operator<(const GraphKey &o) const {
    return std::tie(op, mask, shape, grid, device, args) <
           std::tie(o.op, o.mask, o.shape, o.grid, o.device, o.args);
  }
};
struct GraphCache {
  std::mutex mu;
  std::map<GraphKey, std::pair<hipGraph_t, hipGraphExec_t>> entries;
};
GraphCache g_graphs;
const size_t kMaxGraphs = 64;

void clear_graphs_locked() {
  for (auto &kv : g_graphs.entries) {
    (void)hipGraphExecDestroy(kv.second.second);
    (void)hipGraphDestroy(kv.second.first);
  }
  g_graphs.entries.clear();
}

int launch_graph(int op, unsigned mask, const hqc::KArgs &a, int grid, hipStream_t st,
                 int shape) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  GraphKey key{op, mask, shape, grid, dev, std::vector<unsigned char>(sizeof a)};
  std::memcpy(key.args.data(), &a, sizeof a);
  std::lock_guard<std::mutex> lk(g_graphs.mu);
  auto it = g_graphs.entries.find(key);
  if (it == g_graphs.entries.end()) {
    if (g_graphs.entries.size() >= kMaxGraphs) clear_graphs_locked();
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    e = hipGraphCreate(&graph, 0);
    if (e != hipSuccess) return hip_fail(e);
    hqc::KArgs copy = a;
    void *params[] = {&copy};
    hipKernelNodeParams np;
    std::memset(&np, 0, sizeof np);
    np.func = const_cast<void *>(hqc::kernel_ptr(op, mask, shape));
    np.gridDim = dim3((unsigned)grid);
    np.blockDim = dim3(64);
    np.sharedMemBytes = (unsigned)hqc::lds_bytes_for(op, mask, shape);
    np.kernelParams = params;
    hipGraphNode_t node;
    e = hipGraphAddKernelNode(&node, graph, nullptr, 0, &np);
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(e);
    }
    it = g_graphs.entries.emplace(key, std::make_pair(graph, exec)).first;
  }
  e = hipGraphLaunch(it->second.second, st);
  if (e != hipSuccess) return hip_fail(e);
  return HQC_OK;
}

// Tuned launch configurations: (device, parameter set, batch-size bucket)
// -> (tile, grid), filled by hqc_tune_set / hqc_autotune_decrypt.  The
// bucket of a count is the exponent of the power of two at or above it.
struct TunedEntry {
  int tile, grid, shape;  // shape: 0 or 1 (the kernel shape itself)
};
struct Tuned {
  std::mutex mu;
  std::map<std::tuple<int, int, int>, TunedEntry> table;
};
Tuned g_tuned;

int count_bucket(uint64_t count) {
  int b = 0;
  while (b < 63 && (1ull << b) < count) ++b;
  return b;
}

// current device, or -1 where there is none (the table still works)
int device_or_none() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return -1;
  }
  return dev;
}

bool tuned_lookup(int pid, uint64_t count, int *tile, int *grid, int *shape) {
  const auto key = std::make_tuple(device_or_none(), pid, count_bucket(count));
  std::lock_guard<std::mutex> lk(g_tuned.mu);
  auto it = g_tuned.table.find(key);
  if (it == g_tuned.table.end()) return false;
  *tile = it->second.tile;
  *grid = it->second.grid;
  *shape = it->second.shape;
  return true;
}

// Relative time per item of the sets in the shape-A kernels, as in the
// mixed-set kernels (HQC-1 = 64), from single-set launches on MI355X:
// decryption (and keyed decryption) of 65,536 items at two wavefronts per
// SIMD (0.349 / 0.780 / 1.467 ms), decoding of 262,144 words in the decoding
// layout (0.387 / 0.646 / 1.220 ms).
uint32_t set_cost(int op, int pid) {
  const bool dec = op == hqc::OP_DECODE;
  switch (pid) {
    case 1: return 64;
    case 3: return dec ? 107 : 143;
    case 5: return dec ? 202 : 269;
    default: return 64;
  }
}

// Items of a launch in HQC-1 units of work (the cost-weighted count when
// several sets are present).
uint64_t weighted_items(int op, const hqc::KArgs &a) {
  uint64_t w = 0, nonempty = 0, plain = 0;
  for (uint32_t s = 0; s < a.nseg; ++s) {
    plain += a.seg[s].count;
    w += (uint64_t)a.seg[s].count * set_cost(op, a.seg[s].pid) / 64;
    nonempty += a.seg[s].count > 0;
  }
  return nonempty > 1 ? w : plain;
}

// Splits the segments into tiles; returns the tile count.  With one set,
// tiles of `tile` items.  With several, `tile` is the HQC-1 tile and the
// other sets' tiles are scaled down by their cost per item, to the nearest
// power of two (whole Reed-Solomon passes of 16 or 32 words), so that the
// tiles of the launch take about the same time and the workgroups, which
// take tiles round-robin, finish together -- but not below 4 items (or
// `tile`, if smaller): a tile's fixed cost (loads before the pipeline
// fills, a Reed-Solomon pass) outweighs the balance below that.  Measured
// against unscaled tiles: 65,536 ciphertexts 50/30/20 % HQC-1/3/5 0.90 vs
// 1.28 ms, 1,048,576 decoder words 3.94 vs 4.07 ms.
uint32_t assign_tiles(int op, hqc::KArgs &a, uint32_t tile) {
  uint32_t nonempty = 0;
  for (uint32_t s = 0; s < a.nseg; ++s) nonempty += a.seg[s].count > 0;
  const uint32_t floor_tile = tile < 4 ? tile : 4;
  uint32_t t = 0;
  for (uint32_t s = 0; s < a.nseg; ++s) {
    hqc::SegDev &sg = a.seg[s];
    uint32_t ts = tile;
    if (nonempty > 1) {
      const uint32_t c = set_cost(op, sg.pid);
      const long e = std::lround(std::log2((double)tile * 64.0 / (double)c));
      ts = e <= 0 ? 1u : e >= 6 ? 64u : (1u << e);
      ts = ts < floor_tile ? floor_tile : ts;
    }
    sg.tile = ts;
    sg.first = t;
    t += (sg.count + ts - 1) / ts;
  }
  a.total = t;
  return t;
}

// The launch of `items` items: the caller's shape, tile and grid where set,
// else the tuned table's entry (single-set calls that leave all three open),
// else the built-in choice.  shape out: 0 (A) or 1 (B).
int resolve_launch(int op, const hqc_params_t *p, unsigned mask, uint64_t items, int *shape_out,
                   uint32_t *tile_out, int *grid_out) {
  int grid = p->grid;
  uint32_t tile = (uint32_t)p->tile;
  int shape = p->shape - 1;
  if (shape == 1 && !hqc::shape_exists(op, mask, 1)) return HQC_EINVAL;
  if (grid <= 0 && tile == 0 && p->shape == 0 && (mask == 1u || mask == 2u || mask == 4u)) {
    int tt = 0, tg = 0, ts = 0;
    if (tuned_lookup(mask == 1u ? 1 : mask == 2u ? 3 : 5, items, &tt, &tg, &ts) &&
        hqc::shape_exists(op, mask, ts)) {
      tile = (uint32_t)tt;
      grid = tg;
      shape = ts;
    }
  }
  const int rc = hqc::builtin_launch(op, mask, items, &shape, &tile, &grid);
  if (rc) return rc;
  *shape_out = shape;
  *tile_out = tile;
  *grid_out = grid;
  return HQC_OK;
}

int run(int op, const hqc_params_t *p, hqc::KArgs &a, unsigned mask) {
  hipStream_t st = (hipStream_t)p->stream;
  uint64_t items = 0;
  for (uint32_t s = 0; s < a.nseg; ++s) items += a.seg[s].count;
  if (items == 0) return HQC_OK;
  int grid = 0, shape = 0;
  uint32_t tile = 0;
  {
    const int rc = resolve_launch(op, p, mask, weighted_items(op, a), &shape, &tile, &grid);
    if (rc) return rc;
  }
  assign_tiles(op, a, tile);
  if ((uint32_t)grid > a.total) grid = (int)a.total;
  if (p->flags & HQC_F_PER_ITEM_LAUNCH) {
    // Baseline mode: the same kernel, one launch per item (count = 1).
    for (uint32_t s = 0; s < a.nseg; ++s) {
      const hqc::SegDev &sg = a.seg[s];
      hqc::SetInfo si;
      hqc::set_info(sg.pid, &si);
      for (uint32_t i = 0; i < sg.count; ++i) {
        hqc::KArgs one;
        std::memset(&one, 0, sizeof one);
        one.nseg = 1;
        one.total = 1;
        hqc::SegDev &o = one.seg[0];
        o = sg;
        o.first = 0;
        o.tile = 1;
        o.count = 1;
        const size_t in_words = op == hqc::OP_DECODE ? (size_t)si.v_words : (size_t)si.u_words;
        o.u = sg.u + (size_t)i * in_words;
        if (sg.v) o.v = sg.v + (size_t)i * si.v_words;
        if (sg.y) o.y = sg.y + (size_t)i * si.w;
        if (sg.key_ids) o.key_ids = sg.key_ids + i;
        o.m = sg.m + (size_t)i * si.k;
        hipError_t e = hqc::launch(op, (unsigned)pid_bit(sg.pid), one, 1, st, 0);
        if (e != hipSuccess) return hip_fail(e);
      }
    }
    return HQC_OK;
  }
  if (p->flags & HQC_F_GRAPH) return launch_graph(op, mask, a, grid, st, shape);
  hipError_t e = hqc::launch(op, mask, a, grid, st, shape);
  if (e != hipSuccess) return hip_fail(e);
  return HQC_OK;
}

int check_params(const hqc_params_t *p) {
  if (!p || p->tile < 0 || p->tile > 64) return HQC_EINVAL;
  if (p->shape < 0 || p->shape > 2) return HQC_EINVAL;
  if (p->flags & ~(HQC_F_PER_ITEM_LAUNCH | HQC_F_GRAPH)) return HQC_EINVAL;
  if ((p->flags & HQC_F_PER_ITEM_LAUNCH) && (p->flags & HQC_F_GRAPH)) return HQC_EINVAL;
  if (p->grid < 0) return HQC_EINVAL;
  return HQC_OK;
}

// Validates one segment and fills its device descriptor.  Keyed segments
// carry their key ids (count uint32) in s.y.  out_checked: m_out is memory
// the library itself provides (sized already), not a caller's allocation.
int fill_segment(int op, const hqc_segment_t &s, hqc::SegDev *o, bool out_checked = false) {
  hqc::SetInfo si;
  if (!hqc::set_info(s.param_id, &si) || s.reserved != 0) return HQC_EINVAL;
  if (s.count > HQC_MAX_COUNT) return HQC_ERANGE;
  std::memset(o, 0, sizeof *o);
  o->pid = s.param_id;
  o->count = (uint32_t)s.count;
  if (s.count == 0) return HQC_OK;
  const size_t c = s.count;
  const uint32_t *key_ids = op == hqc::OP_KEYED ? s.y : nullptr;
  if (!s.u || !s.m_out || !aligned(s.u, 8) || !aligned(s.m_out, 4)) return HQC_EINVAL;
  if (op == hqc::OP_DECODE) {
    if (!in_device_allocation(s.u, c * si.v_words * 8)) return HQC_EINVAL;
  } else {
    if (!s.v || !aligned(s.v, 8)) return HQC_EINVAL;
    if (!in_device_allocation(s.u, c * si.u_words * 8)) return HQC_EINVAL;
    if (!in_device_allocation(s.v, c * si.v_words * 8)) return HQC_EINVAL;
    if (op == hqc::OP_DECRYPT || op == hqc::OP_DEBUG) {
      if (!s.y || !aligned(s.y, 4) || !in_device_allocation(s.y, c * si.w * 4)) return HQC_EINVAL;
    } else {
      if (!key_ids || !aligned(key_ids, 4) || !in_device_allocation(key_ids, c * 4))
        return HQC_EINVAL;
    }
  }
  if (!out_checked && !in_device_allocation(s.m_out, c * si.k)) return HQC_EINVAL;
  o->u = s.u;
  o->v = s.v;
  o->y = op == hqc::OP_KEYED ? nullptr : s.y;
  o->key_ids = key_ids;
  o->m = s.m_out;
  return HQC_OK;
}

int run_segments(int op, const hqc_params_t *p, const hqc_segment_t *segs, int nseg,
                 const hqc_keystore_t *ks, uint8_t *dbg = nullptr, bool out_checked = false);

}  // namespace

namespace hqc {
int occupancy_grid(int op, unsigned mask, int shape, int *out) {
  return default_grid(op, mask, out, shape);
}

// The library's built-in launches of single-set decryption on MI355X: the
// autotuner's choices (hqc_autotune_decrypt: 7 rounds in shuffled order,
// four back-to-back graph launches per sample, every candidate's messages
// identical) at each power-of-two batch from 2^8 to 2^20 items: shape
// (1 = A, 2 = B), tile, and the grid in workgroups per compute unit.  A
// batch uses the entry of its bucket (the power of two at or above its
// size; 2^8 below, 2^20 above).
struct BuiltinEntry {
  uint8_t shape, tile, wg_per_cu;
};
constexpr int kBuiltinLo = 8, kBuiltinHi = 20;
constexpr BuiltinEntry kBuiltin[3][kBuiltinHi - kBuiltinLo + 1] = {
    // HQC-1
    {{1, 1, 1}, {1, 1, 12}, {1, 1, 12}, {1, 2, 4}, {1, 4, 4}, {1, 4, 6}, {1, 2, 12},
     {2, 8, 12}, {2, 16, 12}, {2, 32, 12}, {1, 64, 12}, {1, 64, 12}, {2, 64, 12}},
    // HQC-3
    {{2, 1, 1}, {2, 1, 2}, {2, 1, 4}, {2, 2, 4}, {1, 2, 8}, {1, 4, 8}, {2, 4, 12},
     {2, 8, 12}, {2, 16, 12}, {2, 16, 12}, {2, 32, 12}, {2, 64, 12}, {1, 64, 8}},
    // HQC-5
    {{1, 1, 8}, {1, 1, 2}, {1, 1, 8}, {1, 1, 4}, {1, 2, 8}, {1, 4, 8}, {1, 2, 8},
     {1, 4, 8}, {1, 16, 8}, {1, 32, 8}, {1, 64, 8}, {1, 64, 8}, {1, 64, 8}},
};

// The built-in launch of `items` items; only what the caller left open is
// chosen (shape < 0, grid <= 0, tile 0):
//  * single-set decryption (plain or keyed) with all three open: the table
//    above, the grid capped at the shape's occupancy grid;
//  * otherwise shape 1 (three wavefronts per SIMD) for single-set HQC-3
//    once the batch gives its occupancy grid tiles of 16 items, else shape
//    0; the occupancy grid; and the largest power-of-two tile not above
//    items / grid, at most 64.
int builtin_launch(int op, unsigned mask, uint64_t items, int *shape, uint32_t *tile,
                   int *grid) {
  const int set = mask == 1u ? 0 : mask == 2u ? 1 : mask == 4u ? 2 : -1;
  if (set >= 0 && (op == OP_DECRYPT || op == OP_KEYED) && *shape < 0 && *grid <= 0 &&
      *tile == 0) {
    int b = count_bucket(items);
    b = b < kBuiltinLo ? kBuiltinLo : b > kBuiltinHi ? kBuiltinHi : b;
    const BuiltinEntry &e = kBuiltin[set][b - kBuiltinLo];
    if (shape_exists(op, mask, e.shape - 1)) {
      int full = 0, cus = 0;
      int rc = default_grid(op, mask, &full, e.shape - 1, &cus);
      if (rc) return rc;
      *shape = e.shape - 1;
      *tile = e.tile;
      *grid = cus * (int)e.wg_per_cu < full ? cus * (int)e.wg_per_cu : full;
      return HQC_OK;
    }
  }
  if (*shape < 0) {
    *shape = 0;
    if (mask == 2u && shape_exists(op, mask, 1)) {
      int g1 = 0;
      const int rc = default_grid(op, mask, &g1, 1);
      if (rc) return rc;
      if (items >= 16ull * (uint64_t)g1) *shape = 1;
    }
  }
  if (*grid <= 0) {
    const int rc = default_grid(op, mask, grid, *shape);
    if (rc) return rc;
  }
  if (*tile == 0) {
    const uint64_t per = items / (uint64_t)*grid;
    uint32_t t = 1;
    while (t < 64 && 2ull * t <= per) t *= 2;
    *tile = t;
  }
  return HQC_OK;
}
}  // namespace hqc

struct hqc_keystore {
  size_t cap[3];
  uint32_t *y[3];
  unsigned long long *bad;
  int device;
};

namespace {

int run_segments(int op, const hqc_params_t *p, const hqc_segment_t *segs, int nseg,
                 const hqc_keystore_t *ks, uint8_t *dbg, bool out_checked) {
  int rc = check_params(p);
  if (rc) return rc;
  if (!segs || nseg < 1 || nseg > 3) return HQC_EINVAL;
  if (op == hqc::OP_KEYED && !ks) return HQC_EINVAL;
  hqc::KArgs a;
  std::memset(&a, 0, sizeof a);
  unsigned mask = 0, seen = 0;
  uint64_t total = 0;
  for (int i = 0; i < nseg; ++i) {
    if (seen & (unsigned)pid_bit(segs[i].param_id)) return HQC_EINVAL;  // one per set
    seen |= (unsigned)pid_bit(segs[i].param_id);
    hqc::SegDev sd;
    rc = fill_segment(op, segs[i], &sd, out_checked);
    if (rc) return rc;
    if (sd.count == 0) continue;
    if (op == hqc::OP_KEYED) {
      int slot = segs[i].param_id == 1 ? 0 : segs[i].param_id == 3 ? 1 : 2;
      sd.ks_y = ks->y[slot];
      sd.ks_cap = (uint32_t)ks->cap[slot];
      sd.ks_bad = ks->bad;
    }
    mask |= (unsigned)pid_bit(segs[i].param_id);
    total += sd.count;
    sd.dbg = dbg;  // only single-segment debug launches pass one
    a.seg[a.nseg++] = sd;
  }
  if (total > HQC_MAX_COUNT) return HQC_ERANGE;
  if (total == 0) return HQC_OK;
  return run(op, p, a, mask);
}

}  // namespace

extern "C" {

int hqc_sizes(int param_id, hqc_sizes_t *out) {
  hqc::SetInfo si;
  if (!out || !hqc::set_info(param_id, &si)) return HQC_EINVAL;
  out->param_id = param_id;
  out->n = si.n;
  out->n1 = si.n1;
  out->k = si.k;
  out->delta = si.delta;
  out->n2 = si.n2;
  out->mult = si.mult;
  out->w = si.w;
  // encryption-side weights (Table I), reported for completeness
  out->wr = out->we = param_id == 1 ? 75 : param_id == 3 ? 114 : 149;
  out->u_words = si.u_words;
  out->v_words = si.v_words;
  return HQC_OK;
}

int hqc_decrypt_batch(const hqc_params_t *params, const uint64_t *u, const uint64_t *v,
                      const uint32_t *y, uint8_t *m_out, size_t count) {
  if (!params) return HQC_EINVAL;
  hqc_segment_t s;
  std::memset(&s, 0, sizeof s);
  s.param_id = params->param_id;
  s.count = count;
  s.u = u;
  s.v = v;
  s.y = y;
  s.m_out = m_out;
  return run_segments(hqc::OP_DECRYPT, params, &s, 1, nullptr);
}

size_t hqc_debug_bytes(int param_id) {
  hqc::SetInfo si;
  return hqc::set_info(param_id, &si) ? si.dbg_bytes : 0;
}

int hqc_decrypt_debug(const hqc_params_t *params, const uint64_t *u, const uint64_t *v,
                      const uint32_t *y, uint8_t *m_out, uint8_t *dbg_out, size_t count) {
  if (!params || (params->flags & HQC_F_PER_ITEM_LAUNCH)) return HQC_EINVAL;
  hqc::SetInfo si;
  if (!hqc::set_info(params->param_id, &si)) return HQC_EINVAL;
  if (count > HQC_MAX_COUNT) return HQC_ERANGE;
  if (count && (!dbg_out || !aligned(dbg_out, 4) ||
                !in_device_allocation(dbg_out, count * si.dbg_bytes)))
    return HQC_EINVAL;
  hqc_segment_t s;
  std::memset(&s, 0, sizeof s);
  s.param_id = params->param_id;
  s.count = count;
  s.u = u;
  s.v = v;
  s.y = y;
  s.m_out = m_out;
  return run_segments(hqc::OP_DEBUG, params, &s, 1, nullptr, dbg_out);
}

int hqc_decode_batch(const hqc_params_t *params, const uint64_t *r, uint8_t *m_out,
                     size_t count) {
  if (!params) return HQC_EINVAL;
  hqc_segment_t s;
  std::memset(&s, 0, sizeof s);
  s.param_id = params->param_id;
  s.count = count;
  s.u = r;
  s.m_out = m_out;
  return run_segments(hqc::OP_DECODE, params, &s, 1, nullptr);
}

int hqc_decrypt_mixed(const hqc_params_t *params, const hqc_segment_t *segs, int nseg) {
  return run_segments(hqc::OP_DECRYPT, params, segs, nseg, nullptr);
}

int hqc_decode_mixed(const hqc_params_t *params, const hqc_segment_t *segs, int nseg) {
  if (segs)
    for (int i = 0; i < nseg && i < 3; ++i)
      if (segs[i].v || segs[i].y) return HQC_EINVAL;
  return run_segments(hqc::OP_DECODE, params, segs, nseg, nullptr);
}

int hqc_keystore_create(hqc_keystore_t **ks, const size_t cap[3]) {
  if (!ks || !cap) return HQC_EINVAL;
  *ks = nullptr;
  for (int i = 0; i < 3; ++i)
    if (cap[i] > 0xFFFFFFFFull) return HQC_ERANGE;
  hqc_keystore *k = new (std::nothrow) hqc_keystore;
  if (!k) return HQC_ENOMEM;
  std::memset(k, 0, sizeof *k);
  hipError_t e = hipGetDevice(&k->device);
  if (e != hipSuccess) {
    delete k;
    return hip_fail(e);
  }
  const int pids[3] = {1, 3, 5};
  for (int i = 0; i < 3; ++i) {
    hqc::SetInfo si;
    hqc::set_info(pids[i], &si);
    k->cap[i] = cap[i];
    size_t bytes = (cap[i] ? cap[i] : 1) * (size_t)si.w * 4;
    e = hipMalloc(&k->y[i], bytes);
    if (e == hipSuccess) e = hipMemset(k->y[i], 0, bytes);
    if (e != hipSuccess) {
      hqc_keystore_destroy(k);
      return e == hipErrorOutOfMemory ? HQC_ENOMEM : hip_fail(e);
    }
  }
  e = hipMalloc(&k->bad, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(k->bad, 0, sizeof(unsigned long long));
  if (e != hipSuccess) {
    hqc_keystore_destroy(k);
    return hip_fail(e);
  }
  *ks = k;
  return HQC_OK;
}

int hqc_keystore_put_many(hqc_keystore_t *ks, int param_id, uint32_t key_id0, size_t count,
                          const uint32_t *y_host) {
  hqc::SetInfo si;
  if (!ks || !hqc::set_info(param_id, &si)) return HQC_EINVAL;
  if (count == 0) return HQC_OK;
  if (!y_host) return HQC_EINVAL;
  const int slot = param_id == 1 ? 0 : param_id == 3 ? 1 : 2;
  if ((size_t)key_id0 + count > ks->cap[slot]) return HQC_ERANGE;
  std::vector<uint8_t> seen((size_t)si.n);
  for (size_t i = 0; i < count; ++i) {
    const uint32_t *yy = y_host + i * si.w;
    for (int j = 0; j < si.w; ++j) {
      if (yy[j] >= (uint32_t)si.n || seen[yy[j]]) {
        for (int t = 0; t < j; ++t) seen[yy[t]] = 0;
        return HQC_EINVAL;
      }
      seen[yy[j]] = 1;
    }
    for (int j = 0; j < si.w; ++j) seen[yy[j]] = 0;
  }
  hipError_t e = hipMemcpy(ks->y[slot] + (size_t)key_id0 * si.w, y_host, count * si.w * 4,
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e);
  return HQC_OK;
}

int hqc_keystore_put(hqc_keystore_t *ks, int param_id, uint32_t key_id, const uint32_t *y_host) {
  return hqc_keystore_put_many(ks, param_id, key_id, 1, y_host);
}

int hqc_keystore_destroy(hqc_keystore_t *ks) {
  if (!ks) return HQC_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (ks->y[i]) (void)hipFree(ks->y[i]);
  if (ks->bad) (void)hipFree(ks->bad);
  delete ks;
  return HQC_OK;
}

int hqc_keystore_bad_ids(const hqc_keystore_t *ks, uint64_t *out) {
  if (!ks || !out) return HQC_EINVAL;
  unsigned long long v = 0;
  hipError_t e = hipMemcpy(&v, ks->bad, sizeof v, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e);
  *out = v;
  return HQC_OK;
}

int hqc_decrypt_batch_keyed(const hqc_params_t *params, const hqc_keystore_t *ks,
                            const uint64_t *u, const uint64_t *v, const uint32_t *key_ids,
                            uint8_t *m_out, size_t count) {
  if (!params || !ks) return HQC_EINVAL;
  hqc_segment_t s;
  std::memset(&s, 0, sizeof s);
  s.param_id = params->param_id;
  s.count = count;
  s.u = u;
  s.v = v;
  s.y = key_ids;
  s.m_out = m_out;
  return run_segments(hqc::OP_KEYED, params, &s, 1, ks);
}

int hqc_decrypt_mixed_keyed(const hqc_params_t *params, const hqc_keystore_t *ks,
                            const hqc_segment_t *segs, int nseg) {
  if (!ks) return HQC_EINVAL;
  return run_segments(hqc::OP_KEYED, params, segs, nseg, ks);
}

static int run_encrypt(int mode, const hqc_params_t *params, const hqc::EncArgs &a) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  int grid = params->grid;
  if (grid <= 0) {
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, hqc::encrypt_kernel_ptr(mode, params->param_id), 64,
          hqc::encrypt_lds_bytes(params->param_id));
    if (e != hipSuccess) return hip_fail(e);
    grid = cus * (per_cu < 1 ? 1 : per_cu);
  }
  if ((uint32_t)grid > a.count) grid = (int)a.count;
  e = hqc::launch_encrypt(mode, params->param_id, a, grid, (hipStream_t)params->stream);
  if (e != hipSuccess) return hip_fail(e);
  return HQC_OK;
}

int hqc_keygen_batch(const hqc_params_t *params, const uint64_t *h, const uint32_t *x,
                     const uint32_t *y, uint64_t *s_out, size_t count) {
  int rc = check_params(params);
  if (rc) return rc;
  hqc::SetInfo si;
  if (!hqc::set_info(params->param_id, &si)) return HQC_EINVAL;
  if (params->flags) return HQC_EINVAL;
  if (count == 0) return HQC_OK;
  if (count > HQC_MAX_COUNT) return HQC_ERANGE;
  const size_t c = count, uw = (size_t)si.u_words * 8, yw = (size_t)si.w * 4;
  if (!aligned(h, 8) || !aligned(s_out, 8) || !aligned(x, 4) || !aligned(y, 4)) return HQC_EINVAL;
  if (!in_device_allocation(h, c * uw) || !in_device_allocation(s_out, c * uw) ||
      !in_device_allocation(x, c * yw) || !in_device_allocation(y, c * yw))
    return HQC_EINVAL;
  hqc::EncArgs a;
  std::memset(&a, 0, sizeof a);
  a.h = h;
  a.x = x;
  a.y = y;
  a.s_out = s_out;
  a.count = (uint32_t)count;
  return run_encrypt(hqc::ENC_KEYGEN, params, a);
}

int hqc_encrypt_batch(const hqc_params_t *params, const uint64_t *h, const uint64_t *s,
                      const uint8_t *m, const uint32_t *r1, const uint32_t *r2,
                      const uint32_t *e, uint64_t *u_out, uint64_t *v_out, size_t count) {
  int rc = check_params(params);
  if (rc) return rc;
  hqc::SetInfo si;
  if (!hqc::set_info(params->param_id, &si)) return HQC_EINVAL;
  if (params->flags) return HQC_EINVAL;
  if (count == 0) return HQC_OK;
  if (count > HQC_MAX_COUNT) return HQC_ERANGE;
  hqc_sizes_t sz;
  hqc_sizes(params->param_id, &sz);
  const size_t c = count, uw = (size_t)si.u_words * 8, vw = (size_t)si.v_words * 8;
  if (!aligned(h, 8) || !aligned(s, 8) || !aligned(u_out, 8) || !aligned(v_out, 8) ||
      !aligned(r1, 4) || !aligned(r2, 4) || !aligned(e, 4))
    return HQC_EINVAL;
  if (!in_device_allocation(h, c * uw) || !in_device_allocation(s, c * uw) ||
      !in_device_allocation(u_out, c * uw) || !in_device_allocation(v_out, c * vw) ||
      !in_device_allocation(m, c * (size_t)si.k) ||
      !in_device_allocation(r1, c * (size_t)sz.wr * 4) ||
      !in_device_allocation(r2, c * (size_t)sz.wr * 4) ||
      !in_device_allocation(e, c * (size_t)sz.we * 4))
    return HQC_EINVAL;
  hqc::EncArgs a;
  std::memset(&a, 0, sizeof a);
  a.h = h;
  a.s = s;
  a.m = m;
  a.r1 = r1;
  a.r2 = r2;
  a.e = e;
  a.u_out = u_out;
  a.v_out = v_out;
  a.count = (uint32_t)count;
  return run_encrypt(hqc::ENC_ARRAYS, params, a);
}

int hqc_code_encode_batch(const hqc_params_t *params, const uint8_t *m, const uint8_t *sym_err,
                          uint64_t *r_out, size_t count) {
  int rc = check_params(params);
  if (rc) return rc;
  hqc::SetInfo si;
  if (!hqc::set_info(params->param_id, &si)) return HQC_EINVAL;
  if (params->flags) return HQC_EINVAL;
  if (count == 0) return HQC_OK;
  if (count > HQC_MAX_COUNT) return HQC_ERANGE;
  const size_t c = count;
  if (!aligned(r_out, 8) || !in_device_allocation(r_out, c * (size_t)si.v_words * 8) ||
      !in_device_allocation(m, c * (size_t)si.k))
    return HQC_EINVAL;
  if (sym_err && !in_device_allocation(sym_err, c * (size_t)si.n1)) return HQC_EINVAL;
  hqc::EncArgs a;
  std::memset(&a, 0, sizeof a);
  a.m = m;
  a.sym_err = sym_err;
  a.v_out = r_out;
  a.count = (uint32_t)count;
  return run_encrypt(hqc::ENC_CODE, params, a);
}

// ---- KEM -------------------------------------------------------------------------
namespace {

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

struct KemLayout {
  size_t m_off, ok_off, draws_off, total;
};

bool kem_layout(int pid, size_t count, KemLayout *o) {
  hqc::SetInfo si;
  if (!hqc::set_info(pid, &si)) return false;
  o->m_off = 0;
  o->ok_off = round256(count * (size_t)si.k);
  o->draws_off = o->ok_off + round256(count * 4);
  o->total = o->draws_off + count * (size_t)hqc::kem_draw_stride(pid) * 4;
  return true;
}

// shared checks of encaps / decaps; fills si and the workspace layout.
// ws_own: the workspace is the library's own scratch (ws_bytes is its size).
int kem_check(const hqc_params_t *params, const uint64_t *h, const uint64_t *s,
              const uint64_t *u, const uint64_t *v, const uint8_t *key_out, void *ws,
              size_t ws_bytes, size_t count, hqc::SetInfo *si, KemLayout *lay,
              bool ws_own = false) {
  int rc = check_params(params);
  if (rc) return rc;
  if (!hqc::set_info(params->param_id, si)) return HQC_EINVAL;
  if (params->flags) return HQC_EINVAL;
  if (count > HQC_MAX_COUNT) return HQC_ERANGE;
  if (count == 0) return HQC_OK;
  const size_t c = count, uw = (size_t)si->u_words * 8, vw = (size_t)si->v_words * 8;
  if (!aligned(h, 8) || !aligned(s, 8) || !aligned(u, 8) || !aligned(v, 8) ||
      !aligned(key_out, 8) || !aligned(ws, 8))
    return HQC_EINVAL;
  if (!in_device_allocation(h, c * uw) || !in_device_allocation(s, c * uw) ||
      !in_device_allocation(u, c * uw) || !in_device_allocation(v, c * vw) ||
      !in_device_allocation(key_out, c * HQC_KEM_KEY_BYTES))
    return HQC_EINVAL;
  kem_layout(params->param_id, count, lay);
  if (ws_own) return ws_bytes < lay->total ? HQC_ERANGE : HQC_OK;
  if (ws_bytes < lay->total || !in_device_allocation(ws, lay->total)) return HQC_EINVAL;
  return HQC_OK;
}

// Decapsulation (decrypt, draws, re-encryption check, key) with the
// workspace laid out as lay; ws_own as for kem_check.
int kem_decaps(const hqc_params_t *params, const uint64_t *h, const uint64_t *s,
               const uint32_t *y, const uint8_t *sigma, const uint64_t *u, const uint64_t *v,
               uint8_t *key_out, void *workspace, size_t workspace_bytes, size_t count,
               bool ws_own) {
  hqc::SetInfo si;
  KemLayout lay;
  int rc = kem_check(params, h, s, u, v, key_out, workspace, workspace_bytes, count, &si, &lay,
                     ws_own);
  if (rc || count == 0) return rc;
  if (!aligned(y, 4) || !in_device_allocation(y, count * (size_t)si.w * 4)) return HQC_EINVAL;
  if (!aligned(sigma, 8) || !in_device_allocation(sigma, count * (size_t)si.k)) return HQC_EINVAL;
  const int pid = params->param_id;
  hipStream_t st = (hipStream_t)params->stream;
  uint8_t *mp = (uint8_t *)workspace + lay.m_off;
  uint32_t *ok = (uint32_t *)((char *)workspace + lay.ok_off);
  uint32_t *draws = (uint32_t *)((char *)workspace + lay.draws_off);
  // m' = Decrypt(y, (u, v)) into the workspace
  hqc_segment_t sg;
  std::memset(&sg, 0, sizeof sg);
  sg.param_id = pid;
  sg.count = count;
  sg.u = u;
  sg.v = v;
  sg.y = y;
  sg.m_out = mp;
  rc = run_segments(hqc::OP_DECRYPT, params, &sg, 1, nullptr, nullptr, true);
  if (rc) return rc;
  hipError_t e = hqc::launch_kem_draws(pid, mp, draws, (uint32_t)count, st);
  if (e != hipSuccess) return hip_fail(e);
  // re-encrypt m' and compare with (u, v)
  hqc::EncArgs a;
  std::memset(&a, 0, sizeof a);
  a.h = h;
  a.s = s;
  a.m = mp;
  a.draws = draws;
  a.draw_stride = hqc::kem_draw_stride(pid);
  a.u_in = u;
  a.v_in = v;
  a.ok = ok;
  a.count = (uint32_t)count;
  rc = run_encrypt(hqc::ENC_CHECK, params, a);
  if (rc) return rc;
  e = hqc::launch_kem_key(pid, mp, sigma, ok, u, v, key_out, (uint32_t)count, st);
  if (e != hipSuccess) return hip_fail(e);
  return HQC_OK;
}

}  // namespace

int hqc_fixed_weight_batch(const hqc_params_t *params, const uint32_t *draws, uint32_t *supp_out,
                           size_t count) {
  int rc = check_params(params);
  if (rc) return rc;
  hqc::SetInfo si;
  if (!hqc::set_info(params->param_id, &si)) return HQC_EINVAL;
  if (params->flags) return HQC_EINVAL;
  if (count > HQC_MAX_COUNT) return HQC_ERANGE;
  if (count == 0) return HQC_OK;
  const size_t row = hqc::kem_draw_words(params->param_id) * 4;
  if (!aligned(draws, 4) || !aligned(supp_out, 4) || !in_device_allocation(draws, count * row) ||
      !in_device_allocation(supp_out, count * row))
    return HQC_EINVAL;
  hqc::EncArgs a;
  std::memset(&a, 0, sizeof a);
  a.draws = draws;
  a.draw_stride = hqc::kem_draw_words(params->param_id);
  a.supp_out = supp_out;
  a.count = (uint32_t)count;
  return run_encrypt(hqc::ENC_SAMPLE, params, a);
}

size_t hqc_kem_workspace_bytes(int param_id, size_t count) {
  KemLayout lay;
  return kem_layout(param_id, count, &lay) ? lay.total : 0;
}

int hqc_kem_encaps_batch(const hqc_params_t *params, const uint64_t *h, const uint64_t *s,
                         const uint8_t *m, uint64_t *u_out, uint64_t *v_out, uint8_t *key_out,
                         void *workspace, size_t workspace_bytes, size_t count) {
  hqc::SetInfo si;
  KemLayout lay;
  int rc = kem_check(params, h, s, u_out, v_out, key_out, workspace, workspace_bytes, count,
                     &si, &lay);
  if (rc || count == 0) return rc;
  if (!aligned(m, 8) || !in_device_allocation(m, count * (size_t)si.k)) return HQC_EINVAL;
  const int pid = params->param_id;
  hipStream_t st = (hipStream_t)params->stream;
  uint32_t *draws = (uint32_t *)((char *)workspace + lay.draws_off);
  hipError_t e = hqc::launch_kem_draws(pid, m, draws, (uint32_t)count, st);
  if (e != hipSuccess) return hip_fail(e);
  hqc::EncArgs a;
  std::memset(&a, 0, sizeof a);
  a.h = h;
  a.s = s;
  a.m = m;
  a.draws = draws;
  a.draw_stride = hqc::kem_draw_stride(pid);
  a.u_out = u_out;
  a.v_out = v_out;
  a.count = (uint32_t)count;
  rc = run_encrypt(hqc::ENC_STREAM, params, a);
  if (rc) return rc;
  e = hqc::launch_kem_key(pid, m, nullptr, nullptr, u_out, v_out, key_out, (uint32_t)count, st);
  if (e != hipSuccess) return hip_fail(e);
  return HQC_OK;
}

int hqc_kem_decaps_batch(const hqc_params_t *params, const uint64_t *h, const uint64_t *s,
                         const uint32_t *y, const uint8_t *sigma, const uint64_t *u,
                         const uint64_t *v, uint8_t *key_out, void *workspace,
                         size_t workspace_bytes, size_t count) {
  return kem_decaps(params, h, s, y, sigma, u, v, key_out, workspace, workspace_bytes, count,
                    false);
}

int hqc_kem_decaps_batch_noalloc(const hqc_params_t *params, const uint64_t *h,
                                 const uint64_t *s, const uint32_t *y, const uint8_t *sigma,
                                 const uint64_t *u, const uint64_t *v, uint8_t *key_out,
                                 size_t count) {
  if (count == 0) return check_params(params);
  void *scratch = nullptr;
  hipError_t e = hqc::noalloc_scratch(&scratch);
  if (e != hipSuccess) return hip_fail(e);
  return kem_decaps(params, h, s, y, sigma, u, v, key_out, scratch, HQC_NOALLOC_SCRATCH_BYTES,
                    count, true);
}

// ---- adaptive ring multiplication ----------------------------------------------------
size_t hqc_ring_workspace_bytes(int param_id, size_t count, size_t chunk_items) {
  if (count == 0 || chunk_items == 0) return 0;
  return hqc::ring_workspace_bytes(param_id, count, chunk_items);
}

// Measured on MI355X (bench.py --ring-sweep 2048): the sparse path stays
// faster than the dense one up to the sparse list's capacity for every set
// (HQC-1 0.42 vs 0.46 us per item at weight 4096), so the threshold is that
// capacity.
uint32_t hqc_ring_default_threshold(int param_id) {
  switch (param_id) {
    case 1:
    case 3:
    case 5: return HQC_RING_SPARSE_MAX;
    default: return 0;
  }
}

int hqc_ring_mul_batch(const hqc_params_t *params, const uint64_t *a, const uint64_t *b,
                       uint64_t *out, uint8_t *path_out, uint32_t threshold, void *workspace,
                       size_t workspace_bytes, size_t count) {
  int rc = check_params(params);
  if (rc) return rc;
  hqc::SetInfo si;
  if (!hqc::set_info(params->param_id, &si)) return HQC_EINVAL;
  if (params->flags) return HQC_EINVAL;
  if (count > HQC_MAX_COUNT) return HQC_ERANGE;
  if (count == 0) return HQC_OK;
  const size_t c = count, uw = (size_t)si.u_words * 8;
  if (!aligned(a, 8) || !aligned(b, 8) || !aligned(out, 8) || !aligned(workspace, 8))
    return HQC_EINVAL;
  if (!in_device_allocation(a, c * uw) || !in_device_allocation(b, c * uw) ||
      !in_device_allocation(out, c * uw))
    return HQC_EINVAL;
  if (path_out && !in_device_allocation(path_out, c)) return HQC_EINVAL;
  const size_t need = hqc::ring_workspace_bytes(params->param_id, count, 1);
  if (workspace_bytes < need || !in_device_allocation(workspace, workspace_bytes))
    return HQC_EINVAL;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  int grid = params->grid;
  if (grid <= 0) {
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, hqc::ring_sparse_kernel_ptr(params->param_id), 64,
          hqc::ring_sparse_lds(params->param_id));
    if (e != hipSuccess) return hip_fail(e);
    grid = cus * (per_cu < 1 ? 1 : per_cu);
  }
  if ((size_t)grid > count) grid = (int)count;
  e = hqc::launch_ring_mul(params->param_id, a, b, out, path_out, threshold, workspace,
                           workspace_bytes, (uint32_t)count, grid, (hipStream_t)params->stream);
  if (e != hipSuccess) return hip_fail(e);
  return HQC_OK;
}

const char *hqc_strerror(int code) {
  switch (code) {
    case HQC_OK: return "success";
    case HQC_EINVAL: return "invalid argument (pointer, alignment, size, parameter id or flags)";
    case HQC_ERANGE: return "count or key id out of range";
    case HQC_EHIP: return "HIP runtime error (see hqc_last_hip_error)";
    case HQC_ENOMEM: return "out of memory";
    default: return "unknown error code";
  }
}

int hqc_last_hip_error(void) { return g_last_hip; }

int hqc_default_grid(int param_id) {
  unsigned mask = param_id == 0 ? 7u : (unsigned)pid_bit(param_id);
  if (!mask) return HQC_EINVAL;
  int g = 0;
  int rc = default_grid(hqc::OP_DECRYPT, mask, &g);
  return rc ? rc : g;
}

void hqc_shutdown(void) {
  std::lock_guard<std::mutex> lk(g_graphs.mu);
  clear_graphs_locked();
}

int hqc_tune_set(int param_id, size_t count, int tile, int grid, int shape) {
  if (!pid_bit(param_id) || count == 0 || count > HQC_MAX_COUNT) return HQC_EINVAL;
  const bool erase = tile == 0 && grid == 0 && shape == 0;
  if (!erase && (tile < 1 || tile > 64 || grid < 1 || shape < 1 || shape > 2)) return HQC_EINVAL;
  if (shape == 2 && !hqc::shape_exists(hqc::OP_DECRYPT, (unsigned)pid_bit(param_id), 1))
    return HQC_EINVAL;
  const auto key = std::make_tuple(device_or_none(), param_id, count_bucket(count));
  std::lock_guard<std::mutex> lk(g_tuned.mu);
  if (erase)
    g_tuned.table.erase(key);
  else
    g_tuned.table[key] = TunedEntry{tile, grid, shape - 1};
  return HQC_OK;
}

int hqc_tune_get(int param_id, size_t count, int *tile, int *grid, int *shape) {
  if (!pid_bit(param_id) || !tile || !grid || !shape || count == 0 || count > HQC_MAX_COUNT)
    return HQC_EINVAL;
  if (tuned_lookup(param_id, count, tile, grid, shape))
    *shape += 1;
  else
    *tile = *grid = *shape = 0;
  return HQC_OK;
}

int hqc_launch_config(const hqc_params_t *params, size_t count, int *shape, int *tile,
                      int *grid) {
  if (!params || !shape || !tile || !grid || count == 0 || count > HQC_MAX_COUNT) return HQC_EINVAL;
  const int rc = check_params(params);
  if (rc) return rc;
  const unsigned mask = (unsigned)pid_bit(params->param_id);
  if (!mask) return HQC_EINVAL;
  int sh = 0, g = 0;
  uint32_t t = 0;
  const int r2 = resolve_launch(hqc::OP_DECRYPT, params, mask, count, &sh, &t, &g);
  if (r2) return r2;
  const uint64_t tiles = (count + t - 1) / t;
  *shape = sh + 1;
  *tile = (int)t;
  *grid = (uint64_t)g > tiles ? (int)tiles : g;
  return HQC_OK;
}

void hqc_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tuned.mu);
  g_tuned.table.clear();
}

}  // extern "C"
