// hqc_internal.h -- interface between the C ABI (hqc_capi.cpp) and the
// kernels (hqc_kernels.hip).  Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hqc {

// OP_DEBUG is OP_DECRYPT plus stores of each item's intermediates (SegDev::dbg);
// it is a separate kernel so that the other ops carry none of its code.
enum Op : int { OP_DECRYPT = 0, OP_DECODE = 1, OP_KEYED = 2, OP_DEBUG = 3 };

// One homogeneous run of items inside a launch.
struct SegDev {
  const uint64_t *u;        // decrypt: u; decode: received word r
  const uint64_t *v;        // decrypt only
  const uint32_t *y;        // decrypt only (count * w)
  const uint32_t *key_ids;  // keyed only
  const uint32_t *ks_y;     // keyed only: keystore slots of this parameter set
  unsigned long long *ks_bad;  // keyed only: counter of out-of-range key ids
  uint8_t *m;               // count * k
  uint8_t *dbg;             // NULL, or count * SetInfo::dbg_bytes of intermediates
  uint32_t ks_cap;          // keyed only: slots in ks_y
  uint32_t count;
  uint32_t first;           // index of the segment's first tile in the launch
  uint32_t tile;            // items per tile of this segment, 1 .. 64
  int32_t pid;              // 1, 3 or 5
};

// A launch is a list of tiles: up to `tile` consecutive items of one
// segment, decoded by one wavefront.  Segments are stored in tile order
// (seg[s + 1].first follows seg[s]'s last tile) and hold distinct sets.
struct KArgs {
  SegDev seg[3];
  uint32_t nseg;
  uint32_t total;  // tiles
};

// Per-parameter sizes as the kernels see them.
struct SetInfo {
  int n, n1, n2, k, delta, w, mult;
  int u_words, v_words;
  size_t lds_bytes;  // dynamic LDS one workgroup needs for this set (shape 0)
  // per-item intermediates of a debug launch, at these byte offsets: the
  // received word v + u*y (n1*n2 bits, little-endian dwords), the RM
  // symbols (n1), the syndromes S_1..S_2delta, Lambda (2 delta + 1
  // coefficients, Lambda_0 = 1), the error values at the k
  // message positions
  size_t dbg_bytes, dbg_sym, dbg_s, dbg_lam, dbg_e;
};

bool set_info(int pid, SetInfo *out);

// mask: bit 0 = HQC-1, bit 1 = HQC-3, bit 2 = HQC-5 present in the launch.
// shape: the kernel shape (0, or 1 for single-set HQC-1 / HQC-3 kernels
// other than the debug one); kernel_ptr returns NULL where it does not exist.
const void *kernel_ptr(int op, unsigned mask, int shape);
size_t lds_bytes_for(int op, unsigned mask, int shape);
bool shape_exists(int op, unsigned mask, int shape);
hipError_t launch(int op, unsigned mask, const KArgs &a, int grid, hipStream_t stream,
                  int shape);
// the occupancy grid (CUs x resident workgroups) of a kernel on the current
// device, cached (hqc_capi.cpp)
int occupancy_grid(int op, unsigned mask, int shape, int *out);
// the library's built-in launch of `items` items when the caller and the
// tuned table leave it open: shape (-1 = choose), tile and grid (hqc_capi.cpp)
int builtin_launch(int op, unsigned mask, uint64_t items, int *shape, uint32_t *tile,
                   int *grid);

}  // namespace hqc
