// hqc_internal_enc.h -- interface between the C ABI (hqc_capi.cpp) and the
// key-generation, encryption and KEM kernels (hqc_encrypt.hip, hqc_kem.hip).
// Not installed; not part of the public ABI.
#pragma once

#include "hqc_internal.h"

namespace hqc {

// Key generation (s = x + h*y) and encryption (u, v from h, s, m and the
// supports r1, r2, e), one item per workgroup; per-item rows of every array.
// The supports come from arrays (ENC_ARRAYS) or are sampled from a row of
// 32-bit draws (ENC_STREAM, ENC_CHECK: Floyd's sampling, wr, wr, we draws);
// ENC_CHECK compares the result with (u_in, v_in) instead of storing it and
// writes ok[item] = 1 when every word is equal, else 0.  ENC_SAMPLE only
// samples the supports from the draws and stores them.  ENC_CODE only
// encodes: v_out = the concatenated codeword of (the RS codeword of m) +
// sym_err (count rows of n1 bytes; NULL: none).
enum EncMode : int {
  ENC_KEYGEN = 0, ENC_ARRAYS = 1, ENC_STREAM = 2, ENC_CHECK = 3, ENC_SAMPLE = 4, ENC_CODE = 5
};
struct EncArgs {
  const uint64_t *h, *s;
  const uint32_t *x, *y;
  const uint8_t *m;
  const uint32_t *r1, *r2, *e;
  const uint32_t *draws;        // ENC_STREAM / ENC_CHECK: count rows of draw_stride words
  const uint64_t *u_in, *v_in;  // ENC_CHECK
  uint64_t *s_out, *u_out, *v_out;
  uint32_t *ok;                 // ENC_CHECK
  uint32_t *supp_out;           // ENC_SAMPLE: rows of 2 wr + we indices (r1, r2, e)
  const uint8_t *sym_err;       // ENC_CODE: NULL or count rows of n1 bytes
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
// The device address, on the current device, of the library's fixed scratch
// array (HQC_NOALLOC_SCRATCH_BYTES bytes, hqc_kem.hip), looked up once per
// device; every caller on a device shares it.
hipError_t noalloc_scratch(void **ptr);

// Adaptive ring multiplication (hqc_ring.hip).  Workspace: a header for
// count items, then the dense scratch of chunk_items items.
size_t ring_workspace_bytes(int pid, size_t count, size_t chunk_items);
size_t ring_sparse_lds(int pid);
const void *ring_sparse_kernel_ptr(int pid);
hipError_t launch_ring_mul(int pid, const uint64_t *a, const uint64_t *b, uint64_t *out,
                           uint8_t *path_out, uint32_t threshold, void *ws, size_t ws_bytes,
                           uint32_t count, int grid, hipStream_t stream);

}  // namespace hqc
