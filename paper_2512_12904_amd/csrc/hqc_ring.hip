// hqc_ring.hip -- adaptive ring multiplication in GF(2)[X]/(X^n - 1)
// (Sec. III-B, threshold-aware scheduling) for batches of dense operands:
// per item, the Hamming weight of a selects
//   - the sparse path of Eq. (1) when weight(a) <= threshold: the support of
//     a is compacted into LDS and the product is the XOR of windows of a
//     bit-level doubled copy of b, one funnel shift per output dword per
//     index (the decryption kernel's product with a run-time index count);
//   - the dense path otherwise: Karatsuba over 64-bit words (the two-way
//     case of the Toom-Cook family the paper names) down to leaf blocks of M
//     words, leaf products bit by bit, recombination level by level, then
//     reduction mod X^n - 1.
//
// Dense layout: operands padded to W = 2^L M words.  Leaf l (0 <= l < 3^L)
// has base-3 digits d_1 .. d_L (d_1 most significant, the top split); at
// level k digit 0 takes the lower half, 1 the upper half, 2 their sum, so
// its operand is the XOR of the M-word blocks j whose bit L-k is allowed by
// d_k.  Node v of level k has children 3v, 3v+1, 3v+2 (P0, P1, P2) and is
// P0 + X^(64h)(P0 + P1 + P2) + X^(128h) P1, h = M 2^(L-k-1) words.
//
// The path depends on the weight of a, and the sparse path's LDS writes on
// its support: this entry point is for operands whose weight and support are
// not secret (the PKE and KEM entry points take supports directly and run
// in constant time).
#include "hqc_gpu.h"
#include "hqc_device.h"
#include "hqc_internal_enc.h"

namespace hqc {
namespace {

template <int ID> struct RingGeo {
  static constexpr int U = Geo<ID>::U_WORDS;
  static constexpr int L = [] {
    int l = 0;
    while ((U + (1 << l) - 1) >> l > 8) ++l;
    return l;
  }();
  static constexpr int M = (U + (1 << L) - 1) >> L;  // leaf words
  static constexpr int W = M << L;                   // padded operand words
  static constexpr int LEAVES = [] {
    int p = 1;
    for (int i = 0; i < L; ++i) p *= 3;
    return p;
  }();
  static constexpr size_t BUF0 = (size_t)LEAVES * 2 * M;   // leaf products (words)
  static constexpr size_t BUF1 = (size_t)LEAVES / 3 * 4 * M;  // level L-1 results
  static constexpr size_t PER_ITEM = 8 * (BUF0 + BUF1);     // bytes of dense scratch
};

__global__ void ring_init_kernel(uint32_t *ndense) { *ndense = 0u; }

// ---- per-item weight and path --------------------------------------------------
template <int ID>
__global__ __launch_bounds__(64) void ring_weight_kernel(const uint64_t *a, uint32_t threshold,
                                                         uint32_t *path, uint8_t *path_out,
                                                         uint32_t *ndense, uint32_t *dense_list,
                                                         uint32_t count) {
  using G = Geo<ID>;
  const uint32_t item = blockIdx.x;
  if (item >= count) return;
  const int lane = lane_id();
  const uint32_t *row = (const uint32_t *)(a + (size_t)item * G::U_WORDS);
  uint32_t w = 0;
  for (int d = lane; d <= G::DW; d += 64) {
    const uint32_t x = d < G::DW ? row[d] : row[d] & ((1u << G::NB) - 1u);
    w += (uint32_t)__builtin_popcount(x);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) w += (uint32_t)__shfl_xor((int)w, off);
  const uint32_t dense = (w > threshold || w > HQC_RING_SPARSE_MAX) ? 1u : 0u;
  if (lane == 0) {
    path[item] = dense;
    if (path_out) path_out[item] = (uint8_t)dense;
    if (dense) dense_list[atomicAdd(ndense, 1u)] = item;
  }
}

// ---- sparse path ----------------------------------------------------------------
template <int ID>
__global__ __launch_bounds__(64) void ring_sparse_kernel(const uint64_t *a, const uint64_t *b,
                                                         uint64_t *out, const uint32_t *path,
                                                         uint32_t count) {
  using G = Geo<ID>;
  extern __shared__ uint32_t lds[];
  uint32_t *u2 = lds;
  uint32_t *list = lds + G::U2;
  const int lane = lane_id();
  for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
    if (path[item] != 0u) continue;  // uniform: one item per wavefront
    // the doubled copy of b
    const uint32_t *brow = (const uint32_t *)(b + (size_t)item * G::U_WORDS);
    for (int d = lane; d <= G::DW; d += 64) u2[d] = brow[d];
    build_doubled<ID>(u2);
    // the support of a, in increasing order: lane l owns dwords l, l + 64, ...
    const uint32_t *arow = (const uint32_t *)(a + (size_t)item * G::U_WORDS);
    uint32_t base = 0;
    for (int d0 = 0; d0 <= G::DW; d0 += 64) {
      const int d = d0 + lane;
      const uint32_t raw = arow[d <= G::DW ? d : G::DW];
      uint32_t x = d < G::DW ? raw : (d == G::DW ? raw & ((1u << G::NB) - 1u) : 0u);
      const uint32_t c = (uint32_t)__builtin_popcount(x);
      uint32_t pre = c;  // inclusive scan over the lanes
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)pre, off);
        if (lane >= off) pre += t;
      }
      uint32_t at = base + pre - c;
      while (x) {
        list[at++] = 32u * (uint32_t)d + (uint32_t)__builtin_ctz(x);
        x &= x - 1u;
      }
      base += rdlane(pre, 63);
    }
    wave_sync();
    // XOR of windows: output dword lane * R + j
    uint32_t acc[G::R];
#pragma unroll
    for (int j = 0; j < G::R; ++j) acc[j] = 0;
    const uint32_t *wb = u2 + lane * G::R;
    for (uint32_t k0 = 0; k0 < base; k0 += 64) {
      const uint32_t idx = k0 + (uint32_t)lane < base ? list[k0 + lane] : 0u;
      const uint32_t sh = (uint32_t)G::n - idx;  // idx < n: shift in [1, n]
      const int cnt = base - k0 < 64u ? (int)(base - k0) : 64;
      for (int kk = 0; kk < cnt; ++kk) {
        const uint32_t s = rdlane(sh, kk);
        const uint32_t *p = wb + (s >> 5);
        const uint32_t r = s & 31u;
        uint32_t lo = p[0];
#pragma unroll
        for (int j = 0; j < G::R; ++j) {
          const uint32_t hi = p[j + 1];
          acc[j] ^= __builtin_amdgcn_alignbit(hi, lo, r);
          lo = hi;
        }
      }
    }
    uint32_t *dst = (uint32_t *)(out + (size_t)item * G::U_WORDS);
#pragma unroll
    for (int j = 0; j < G::R; ++j) {
      const int d = lane * G::R + j;
      if (d < 2 * G::U_WORDS)
        dst[d] = d < G::DW ? acc[j] : (d == G::DW ? acc[j] & ((1u << G::NB) - 1u) : 0u);
    }
    wave_sync();
  }
}

// ---- dense path -----------------------------------------------------------------
// word t (0 <= t < W) of the padded operand x with bits >= n cleared
template <int ID> __device__ __forceinline__ uint64_t padded(const uint64_t *row, int t) {
  using G = Geo<ID>;
  constexpr int NW = (G::n + 63) / 64;
  constexpr int REM = G::n % 64;
  if (t >= NW) return 0;
  const uint64_t x = row[t];
  return t == NW - 1 && REM ? x & ((1ull << REM) - 1ull) : x;
}

// one thread per (dense item of the chunk, leaf): operands then the leaf product
template <int ID>
__global__ __launch_bounds__(256) void ring_leaf_kernel(const uint64_t *a, const uint64_t *b,
                                                        const uint32_t *ndense,
                                                        const uint32_t *dense_list,
                                                        uint32_t chunk0, uint32_t chunk,
                                                        uint64_t *buf0) {
  using RG = RingGeo<ID>;
  constexpr int M = RG::M, L = RG::L;
  const uint32_t nd = *ndense;
  const uint32_t nitems = nd > chunk0 ? (nd - chunk0 < chunk ? nd - chunk0 : chunk) : 0u;
  const size_t total = (size_t)nitems * RG::LEAVES;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (size_t)gridDim.x * blockDim.x) {
    const uint32_t slot = (uint32_t)(g / RG::LEAVES), leaf = (uint32_t)(g % RG::LEAVES);
    const uint32_t item = dense_list[chunk0 + slot];
    const uint64_t *ar = a + (size_t)item * Geo<ID>::U_WORDS;
    const uint64_t *br = b + (size_t)item * Geo<ID>::U_WORDS;
    // digits, most significant first; allowed block-bit sets per level
    uint32_t dig[L > 0 ? L : 1];
    uint32_t rest = leaf, twos = 0;
    for (int k = L - 1; k >= 0; --k) {
      dig[k] = rest % 3u;
      rest /= 3u;
    }
    for (int k = 0; k < L; ++k) twos += dig[k] == 2u;
    uint64_t A[M], B[M];
#pragma unroll
    for (int t = 0; t < M; ++t) A[t] = B[t] = 0;
    // every block index j consistent with the digits: bit (L-1-k) of j is
    // dig[k] for digits 0/1, free for digit 2
    for (uint32_t c = 0; c < (1u << twos); ++c) {
      uint32_t j = 0, used = 0;
      for (int k = 0; k < L; ++k) {
        uint32_t bitv = dig[k];
        if (dig[k] == 2u) bitv = (c >> used++) & 1u;
        j = (j << 1) | bitv;
      }
#pragma unroll
      for (int t = 0; t < M; ++t) {
        A[t] ^= padded<ID>(ar, (int)j * M + t);
        B[t] ^= padded<ID>(br, (int)j * M + t);
      }
    }
    // C = A * B, bit by bit over A
    uint64_t C[2 * M];
#pragma unroll
    for (int t = 0; t < 2 * M; ++t) C[t] = 0;
#pragma unroll
    for (int s = 0; s < M; ++s) {
      for (int r = 0; r < 64; ++r) {
        const uint64_t mask = 0ull - ((A[s] >> r) & 1ull);
#pragma unroll
        for (int j = 0; j < M; ++j) {
          C[s + j] ^= (B[j] << r) & mask;
          C[s + j + 1] ^= (r ? B[j] >> (64 - r) : 0ull) & mask;
        }
      }
    }
    uint64_t *dst = buf0 + ((size_t)slot * RG::LEAVES + leaf) * (2 * M);
#pragma unroll
    for (int t = 0; t < 2 * M; ++t) dst[t] = C[t];
  }
}

// level k: nodes v < 3^k of 4h words from children (2h words each) in src
template <int ID>
__global__ __launch_bounds__(256) void ring_combine_kernel(const uint32_t *ndense, uint32_t chunk0,
                                                           uint32_t chunk, const uint64_t *src,
                                                           uint64_t *dst, uint32_t nodes,
                                                           uint32_t h, size_t src_item,
                                                           size_t dst_item) {
  const uint32_t nd = *ndense;
  const uint32_t nitems = nd > chunk0 ? (nd - chunk0 < chunk ? nd - chunk0 : chunk) : 0u;
  const size_t per = (size_t)nodes * 4 * h;
  const size_t total = (size_t)nitems * per;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (size_t)gridDim.x * blockDim.x) {
    const size_t slot = g / per, r = g % per;
    const uint32_t v = (uint32_t)(r / (4 * h)), k = (uint32_t)(r % (4 * h));
    const uint64_t *p0 = src + slot * src_item + (size_t)(3 * v) * 2 * h;
    const uint64_t *p1 = p0 + 2 * h, *p2 = p1 + 2 * h;
    uint64_t x = 0;
    if (k < 2 * h) x ^= p0[k];
    if (k >= h && k < 3 * h) x ^= p0[k - h] ^ p1[k - h] ^ p2[k - h];
    if (k >= 2 * h) x ^= p1[k - 2 * h];
    dst[slot * dst_item + r] = x;
  }
}

// out = C mod (X^n - 1): dword d of out = dword d of C + bits [32d + n, 32d + n + 32) of C
template <int ID>
__global__ __launch_bounds__(256) void ring_fold_kernel(const uint32_t *ndense,
                                                        const uint32_t *dense_list, uint32_t chunk0,
                                                        uint32_t chunk, const uint64_t *cbuf,
                                                        size_t c_item, uint64_t *out) {
  using G = Geo<ID>;
  const uint32_t nd = *ndense;
  const uint32_t nitems = nd > chunk0 ? (nd - chunk0 < chunk ? nd - chunk0 : chunk) : 0u;
  constexpr int ODW = 2 * G::U_WORDS;
  const size_t total = (size_t)nitems * ODW;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (size_t)gridDim.x * blockDim.x) {
    const uint32_t slot = (uint32_t)(g / ODW);
    const int d = (int)(g % ODW);
    const uint32_t item = dense_list[chunk0 + slot];
    const uint32_t *c = (const uint32_t *)(cbuf + slot * c_item);
    uint32_t val = 0;
    if (d <= G::DW) {
      const uint32_t pos = 32u * (uint32_t)d + (uint32_t)G::n;
      const uint32_t q = pos >> 5, r = pos & 31u;
      val = c[d] ^ __builtin_amdgcn_alignbit(c[q + 1], c[q], r);
      if (d == G::DW) val &= (1u << G::NB) - 1u;
    }
    ((uint32_t *)(out + (size_t)item * G::U_WORDS))[d] = val;
  }
}

template <int ID> size_t sparse_lds() { return 4 * ((size_t)Geo<ID>::U2 + HQC_RING_SPARSE_MAX); }

template <int ID>
hipError_t ring_run(const uint64_t *a, const uint64_t *b, uint64_t *out, uint8_t *path_out,
                    uint32_t threshold, uint8_t *ws, size_t ws_bytes, uint32_t count, int grid,
                    hipStream_t st) {
  using RG = RingGeo<ID>;
  // workspace: ndense | path[count] | dense_list[count] | dense scratch (chunks)
  uint32_t *ndense = (uint32_t *)ws;
  uint32_t *path = ndense + 64;
  uint32_t *dense_list = path + count;
  const size_t head = (size_t)4 * (64 + 2 * (size_t)count);
  uint8_t *scratch = ws + (head + 255) / 256 * 256;
  const size_t room = ws_bytes - (size_t)(scratch - ws);
  const uint32_t chunk = (uint32_t)(room / RG::PER_ITEM < count ? room / RG::PER_ITEM : count);
  uint64_t *buf0 = (uint64_t *)scratch;
  uint64_t *buf1 = buf0 + (size_t)chunk * RG::BUF0;

  ring_init_kernel<<<dim3(1), dim3(1), 0, st>>>(ndense);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  ring_weight_kernel<ID><<<dim3(count), dim3(64), 0, st>>>(a, threshold, path, path_out, ndense,
                                                           dense_list, count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  ring_sparse_kernel<ID><<<dim3((unsigned)grid), dim3(64), sparse_lds<ID>(), st>>>(a, b, out, path,
                                                                                count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned blocks = 2048;
  for (uint32_t c0 = 0; c0 < count; c0 += chunk) {
    ring_leaf_kernel<ID><<<dim3(blocks), dim3(256), 0, st>>>(a, b, ndense, dense_list, c0, chunk, buf0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // levels L-1 .. 0, ping-pong between buf0 and buf1
    const uint64_t *src = buf0;
    uint64_t *dst = buf1;
    size_t src_item = RG::BUF0, dst_item = RG::BUF1;
    uint32_t nodes = RG::LEAVES / 3, h = RG::M;
    for (int k = RG::L - 1; k >= 0; --k) {
      ring_combine_kernel<ID><<<dim3(blocks), dim3(256), 0, st>>>(ndense, c0, chunk, src, dst, nodes,
                                                                 h, src_item, dst_item);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const uint64_t *ns = dst;
      dst = (uint64_t *)src;
      src = ns;
      const size_t t = src_item;
      src_item = dst_item;
      dst_item = t;
      nodes /= 3;
      h *= 2;
    }
    ring_fold_kernel<ID><<<dim3(blocks), dim3(256), 0, st>>>(ndense, dense_list, c0, chunk, src,
                                                             src_item, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

size_t ring_workspace_bytes(int pid, size_t count, size_t chunk_items) {
  const size_t head = (4 * (64 + 2 * count) + 255) / 256 * 256;
  size_t per = 0;
  switch (pid) {
    case 1: per = RingGeo<1>::PER_ITEM; break;
    case 3: per = RingGeo<3>::PER_ITEM; break;
    case 5: per = RingGeo<5>::PER_ITEM; break;
    default: return 0;
  }
  return head + per * (chunk_items < count ? chunk_items : count);
}

size_t ring_sparse_lds(int pid) {
  switch (pid) {
    case 1: return sparse_lds<1>();
    case 3: return sparse_lds<3>();
    default: return sparse_lds<5>();
  }
}

const void *ring_sparse_kernel_ptr(int pid) {
  switch (pid) {
    case 1: return (const void *)&ring_sparse_kernel<1>;
    case 3: return (const void *)&ring_sparse_kernel<3>;
    default: return (const void *)&ring_sparse_kernel<5>;
  }
}

hipError_t launch_ring_mul(int pid, const uint64_t *a, const uint64_t *b, uint64_t *out,
                           uint8_t *path_out, uint32_t threshold, void *ws, size_t ws_bytes,
                           uint32_t count, int grid, hipStream_t stream) {
  switch (pid) {
    case 1: return ring_run<1>(a, b, out, path_out, threshold, (uint8_t *)ws, ws_bytes, count, grid, stream);
    case 3: return ring_run<3>(a, b, out, path_out, threshold, (uint8_t *)ws, ws_bytes, count, grid, stream);
    default: return ring_run<5>(a, b, out, path_out, threshold, (uint8_t *)ws, ws_bytes, count, grid, stream);
  }
}

}  // namespace hqc
