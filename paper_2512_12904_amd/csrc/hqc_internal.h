// hqc_internal.h -- interface between the C ABI (hqc_capi.cpp) and the
// kernels (hqc_kernels.hip).  Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hqc {

enum Op : int { OP_DECRYPT = 0, OP_DECODE = 1, OP_KEYED = 2 };

// One homogeneous run of items inside a launch.
struct SegDev {
  const uint64_t *u;        // decrypt: u; decode: received word r
  const uint64_t *v;        // decrypt only
  const uint32_t *y;        // decrypt only (count * w)
  const uint32_t *key_ids;  // keyed only
  const uint32_t *ks_y;     // keyed only: keystore slots of this parameter set
  unsigned long long *ks_bad;  // keyed only: counter of out-of-range key ids
  uint8_t *m;               // count * k
  uint32_t ks_cap;          // keyed only: slots in ks_y
  uint32_t count;
  uint32_t first;           // index of the segment's first tile in the launch
  int32_t pid;              // 1, 3 or 5
};

// A launch is a list of tiles: up to `tile` consecutive items of one
// segment, decoded by one wavefront.
struct KArgs {
  SegDev seg[3];
  uint32_t nseg;
  uint32_t total;  // tiles
  uint32_t tile;   // items per tile, 1 .. 64
};

// Per-parameter sizes as the kernels see them.
struct SetInfo {
  int n, n1, n2, k, delta, w, mult;
  int u_words, v_words;
  size_t lds_bytes;  // dynamic LDS one workgroup needs for this set
};

bool set_info(int pid, SetInfo *out);

// Key generation (s = x + h*y) and encryption (u, v from h, s, m and the
// supports r1, r2, e), one item per workgroup; per-item rows of every array.
// The supports come from arrays (ENC_ARRAYS) or are sampled from a row of
// 32-bit draws (ENC_STREAM, ENC_CHECK: Floyd's sampling, wr, wr, we draws);
// ENC_CHECK compares the result with (u_in, v_in) instead of storing it and
// writes ok[item] = 1 when every word is equal, else 0.
enum EncMode : int { ENC_KEYGEN = 0, ENC_ARRAYS = 1, ENC_STREAM = 2, ENC_CHECK = 3 };
struct EncArgs {
  const uint64_t *h, *s;
  const uint32_t *x, *y;
  const uint8_t *m;
  const uint32_t *r1, *r2, *e;
  const uint32_t *draws;        // ENC_STREAM / ENC_CHECK: count rows of draw_stride words
  const uint64_t *u_in, *v_in;  // ENC_CHECK
  uint64_t *s_out, *u_out, *v_out;
  uint32_t *ok;                 // ENC_CHECK
  uint32_t draw_stride;
  uint32_t count;
};
const void *encrypt_kernel_ptr(int mode, int pid);
size_t encrypt_lds_bytes(int pid);
hipError_t launch_encrypt(int mode, int pid, const EncArgs &a, int grid, hipStream_t stream);

// SHAKE256 kernels of the KEM, one item per lane.  draw_words(pid) = 2 wr + we
// draws per item; rows of draw_stride(pid) words (whole 136-byte squeeze
// blocks).
uint32_t kem_draw_words(int pid);
uint32_t kem_draw_stride(int pid);
// draws[i] = SHAKE256(m[i] || 0x03)
hipError_t launch_kem_draws(int pid, const uint8_t *m, uint32_t *draws, uint32_t count,
                            hipStream_t stream);
// key[i] = SHAKE256(p[i] || u[i] || v[i] || 0x04)[0, 32) with p[i] = m[i], or,
// when ok != nullptr, p[i] = ok[i] ? m[i] : sigma[i]
hipError_t launch_kem_key(int pid, const uint8_t *m, const uint8_t *sigma, const uint32_t *ok,
                          const uint64_t *u, const uint64_t *v, uint8_t *key, uint32_t count,
                          hipStream_t stream);
// mask: bit 0 = HQC-1, bit 1 = HQC-3, bit 2 = HQC-5 present in the launch.
const void *kernel_ptr(int op, unsigned mask);
size_t lds_bytes_for(unsigned mask);
hipError_t launch(int op, unsigned mask, const KArgs &a, int grid, hipStream_t stream);

}  // namespace hqc
