// hqc_kem.hip -- the SHAKE256 steps of the KEM around HQC.PKE (Sec. II-A:
// domain-separated SHAKE-derived functions for seed formation and key
// derivation), batched with one item per lane.
//
//   draws(m)        = SHAKE256(m || 0x03): the 32-bit draws from which
//                     r1, r2 and e are sampled (2 wr + we words)
//   key(p, u, v)    = SHAKE256(p || u || v || 0x04), first 32 bytes, with u
//                     and v as their little-endian 64-bit words
//
// SHAKE256 is the FIPS 202 sponge over Keccak-f[1600] with a 136-byte rate;
// the message is followed by 0x1F and the rate block ends with 0x80.  The 25
// state lanes live in VGPRs as (lo, hi) dword pairs: rotations are two
// v_alignbit_b32, the chi and theta combinations three-input bit operations
// (v_bitop3_b32).  Every item of a launch has the same length, so all loop
// bounds and branches are uniform; data only flows through the lanes' own
// state and loads at fixed offsets of their own rows.
#include <map>
#include <mutex>
#include <utility>

#include "hqc_device.h"
#include "hqc_gpu.h"
#include "hqc_internal_enc.h"

namespace hqc {
namespace {

struct L64 {
  uint32_t lo, hi;
};

__device__ __forceinline__ L64 ld64(const uint64_t *p) {
  const uint64_t x = *p;
  return {(uint32_t)x, (uint32_t)(x >> 32)};
}

// rotate left by R (compile time), 0 <= R < 64
template <int R> __device__ __forceinline__ L64 rotl(L64 x) {
  if constexpr (R == 0) {
    return x;
  } else if constexpr (R == 32) {
    return {x.hi, x.lo};
  } else if constexpr (R < 32) {
    return {__builtin_amdgcn_alignbit(x.lo, x.hi, 32 - R), __builtin_amdgcn_alignbit(x.hi, x.lo, 32 - R)};
  } else {
    return rotl<R - 32>(L64{x.hi, x.lo});
  }
}

// ---- Keccak-f[1600] constants from FIPS 202's definitions --------------------

// rho offset of lane x + 5y and pi destination of lane x + 5y
struct RhoPi {
  int rho[25];
  int dst[25];
};
constexpr RhoPi make_rho_pi() {
  RhoPi t{};
  t.rho[0] = 0;
  int x = 1, y = 0;
  for (int s = 0; s < 24; ++s) {
    t.rho[x + 5 * y] = ((s + 1) * (s + 2) / 2) % 64;
    const int nx = y, ny = (2 * x + 3 * y) % 5;
    x = nx;
    y = ny;
  }
  // pi: A'[x', y'] = A[x' + 3y', x'], i.e. lane (x, y) moves to (y, 2x + 3y)
  for (int yy = 0; yy < 5; ++yy)
    for (int xx = 0; xx < 5; ++xx) t.dst[xx + 5 * yy] = yy + 5 * ((2 * xx + 3 * yy) % 5);
  return t;
}
constexpr RhoPi kRhoPi = make_rho_pi();

// iota round constants: bit 2^j - 1 of RC[ir] is rc(j + 7 ir), rc the LFSR
// x^8 + x^6 + x^5 + x^4 + 1 read from its first bit
struct RoundConstants {
  uint32_t lo[24], hi[24];
};
constexpr RoundConstants make_round_constants() {
  RoundConstants t{};
  for (int ir = 0; ir < 24; ++ir) {
    unsigned long long rc = 0;
    for (int j = 0; j <= 6; ++j) {
      const int tt = (j + 7 * ir) % 255;
      unsigned r = 1u;
      for (int i = 1; i <= tt; ++i) {
        r <<= 1;
        const unsigned b8 = (r >> 8) & 1u;
        r = (r ^ (b8 | b8 << 4 | b8 << 5 | b8 << 6)) & 0xFFu;
      }
      if (r & 1u) rc |= 1ull << ((1u << j) - 1u);
    }
    t.lo[ir] = (uint32_t)rc;
    t.hi[ir] = (uint32_t)(rc >> 32);
  }
  return t;
}
__constant__ RoundConstants kRC = make_round_constants();

template <int I> __device__ __forceinline__ L64 rot_lane(L64 x) { return rotl<kRhoPi.rho[I]>(x); }

template <int... I>
__device__ __forceinline__ void rho_pi(const L64 (&A)[25], L64 (&B)[25],
                                       std::integer_sequence<int, I...>) {
  ((B[kRhoPi.dst[I]] = rot_lane<I>(A[I])), ...);
}

__device__ __forceinline__ void keccak_f1600(L64 (&A)[25]) {
#pragma unroll 4
  for (int ir = 0; ir < 24; ++ir) {
    // theta
    L64 C[5];
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      C[x].lo = xor3(xor3(A[x].lo, A[x + 5].lo, A[x + 10].lo), A[x + 15].lo, A[x + 20].lo);
      C[x].hi = xor3(xor3(A[x].hi, A[x + 5].hi, A[x + 10].hi), A[x + 15].hi, A[x + 20].hi);
    }
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      const L64 r = rotl<1>(C[(x + 1) % 5]), l = C[(x + 4) % 5];
#pragma unroll
      for (int y = 0; y < 5; ++y) {
        A[x + 5 * y].lo = xor3(A[x + 5 * y].lo, l.lo, r.lo);
        A[x + 5 * y].hi = xor3(A[x + 5 * y].hi, l.hi, r.hi);
      }
    }
    // rho and pi
    L64 B[25];
    rho_pi(A, B, std::make_integer_sequence<int, 25>{});
    // chi
#pragma unroll
    for (int y = 0; y < 5; ++y) {
#pragma unroll
      for (int x = 0; x < 5; ++x) {
        const L64 a = B[x + 5 * y], b = B[(x + 1) % 5 + 5 * y], c = B[(x + 2) % 5 + 5 * y];
        A[x + 5 * y].lo = a.lo ^ (~b.lo & c.lo);
        A[x + 5 * y].hi = a.hi ^ (~b.hi & c.hi);
      }
    }
    // iota
    A[0].lo ^= kRC.lo[ir];
    A[0].hi ^= kRC.hi[ir];
  }
}

constexpr int RATE_WORDS = 17;  // 136-byte rate in 64-bit lanes

// ---- draws(m) = SHAKE256(m || 0x03) ------------------------------------------
template <int ID> struct KemGeo {
  static constexpr int k = Set<ID>::k;
  static constexpr int P = k / 8;                                   // m in 64-bit words
  static constexpr int NDRAW = 2 * Set<ID>::wr + Set<ID>::we;       // 32-bit draws
  static constexpr int SQ = (NDRAW + 2 * RATE_WORDS - 1) / (2 * RATE_WORDS);  // squeeze blocks
  static constexpr int STRIDE = SQ * 2 * RATE_WORDS;                // words per row
  static constexpr int U = Geo<ID>::U_WORDS, V = Geo<ID>::V_WORDS;
  // key input p || u || v || 0x04 in 64-bit words, and its padded blocks
  static constexpr int KBYTES = k + 8 * U + 8 * V + 1;
  static constexpr int KBLOCKS = KBYTES / 136 + 1;
  static_assert(k % 8 == 0 && P + 1 < RATE_WORDS, "m and its suffix fit one block");
};

template <int ID>
__global__ __launch_bounds__(64) void kem_draws_kernel(const uint8_t *m, uint32_t *draws,
                                                       uint32_t count) {
  using K = KemGeo<ID>;
  const uint32_t item = blockIdx.x * 64u + threadIdx.x;
  if (item >= count) return;
  L64 A[25];
#pragma unroll
  for (int i = 0; i < 25; ++i) A[i] = {0u, 0u};
  const uint64_t *mw = (const uint64_t *)(m + (size_t)item * K::k);
#pragma unroll
  for (int i = 0; i < K::P; ++i) A[i] = ld64(mw + i);
  A[K::P].lo ^= 0x03u | 0x1Fu << 8;       // domain byte, then the SHAKE suffix and pad start
  A[RATE_WORDS - 1].hi ^= 0x80u << 24;    // pad end
  keccak_f1600(A);
  uint64_t *out = (uint64_t *)(draws + (size_t)item * K::STRIDE);
#pragma unroll 1
  for (int b = 0; b < K::SQ; ++b) {
    if (b > 0) keccak_f1600(A);
#pragma unroll
    for (int i = 0; i < RATE_WORDS; ++i)
      out[b * RATE_WORDS + i] = (uint64_t)A[i].hi << 32 | A[i].lo;
  }
}

// ---- key = SHAKE256(p || u || v || 0x04)[0, 32) -------------------------------
// word w of the padded key input of this lane's item (w uniform)
template <int ID>
__device__ __forceinline__ L64 key_word(int w, const uint64_t *pre, const uint64_t *alt, bool use_pre,
                                        const uint64_t *u, const uint64_t *v) {
  using K = KemGeo<ID>;
  L64 x = {0u, 0u};
  if (w < K::P) {
    const L64 a = ld64(pre + w), b = ld64(alt + w);
    x = {use_pre ? a.lo : b.lo, use_pre ? a.hi : b.hi};
  } else if (w < K::P + K::U) {
    x = ld64(u + (w - K::P));
  } else if (w < K::P + K::U + K::V) {
    x = ld64(v + (w - K::P - K::U));
  } else if (w == K::P + K::U + K::V) {
    x.lo = 0x04u | 0x1Fu << 8;
  }
  if (w == K::KBLOCKS * RATE_WORDS - 1) x.hi ^= 0x80u << 24;
  return x;
}

template <int ID, bool DECAPS>
__global__ __launch_bounds__(64) void kem_key_kernel(const uint8_t *m, const uint8_t *sigma,
                                                     const uint32_t *ok, const uint64_t *u,
                                                     const uint64_t *v, uint8_t *key,
                                                     uint32_t count) {
  using K = KemGeo<ID>;
  const uint32_t item = blockIdx.x * 64u + threadIdx.x;
  if (item >= count) return;
  const uint64_t *pre = (const uint64_t *)(m + (size_t)item * K::k);
  const uint64_t *alt = DECAPS ? (const uint64_t *)(sigma + (size_t)item * K::k) : pre;
  const bool use_pre = DECAPS ? ok[item] != 0u : true;
  const uint64_t *ur = u + (size_t)item * K::U, *vr = v + (size_t)item * K::V;
  L64 A[25];
#pragma unroll
  for (int i = 0; i < 25; ++i) A[i] = {0u, 0u};
  // the next block's words are loaded while this one is permuted
  L64 nxt[RATE_WORDS];
#pragma unroll
  for (int i = 0; i < RATE_WORDS; ++i) nxt[i] = key_word<ID>(i, pre, alt, use_pre, ur, vr);
#pragma unroll 1
  for (int b = 0; b < K::KBLOCKS; ++b) {
#pragma unroll
    for (int i = 0; i < RATE_WORDS; ++i) {
      A[i].lo ^= nxt[i].lo;
      A[i].hi ^= nxt[i].hi;
    }
    // next block: most lie inside u or inside v (one base, seventeen
    // loads at fixed offsets); the few that straddle a boundary or hold
    // the padding take the word-by-word path (b is uniform: scalar branches)
    const int w0 = (b + 1) * RATE_WORDS;
    constexpr int WU = K::P, WV = K::P + K::U, WE = K::P + K::U + K::V;
    if (w0 >= WU && w0 + RATE_WORDS <= WV) {
      const uint64_t *src = ur + (w0 - WU);
#pragma unroll
      for (int i = 0; i < RATE_WORDS; ++i) nxt[i] = ld64(src + i);
    } else if (w0 >= WV && w0 + RATE_WORDS <= WE) {
      const uint64_t *src = vr + (w0 - WV);
#pragma unroll
      for (int i = 0; i < RATE_WORDS; ++i) nxt[i] = ld64(src + i);
    } else if (b + 1 < K::KBLOCKS) {
#pragma unroll
      for (int i = 0; i < RATE_WORDS; ++i)
        nxt[i] = key_word<ID>(w0 + i, pre, alt, use_pre, ur, vr);
    }
    keccak_f1600(A);
  }
  uint64_t *out = (uint64_t *)(key + (size_t)item * 32);
#pragma unroll
  for (int i = 0; i < 4; ++i) out[i] = (uint64_t)A[i].hi << 32 | A[i].lo;
}

template <int ID> hipError_t draws_for(const uint8_t *m, uint32_t *draws, uint32_t count,
                                       hipStream_t stream) {
  const unsigned blocks = (count + 63u) / 64u;
  kem_draws_kernel<ID><<<dim3(blocks), dim3(64), 0, stream>>>(m, draws, count);
  return hipGetLastError();
}

template <int ID> hipError_t key_for(const uint8_t *m, const uint8_t *sigma, const uint32_t *ok,
                                     const uint64_t *u, const uint64_t *v, uint8_t *key,
                                     uint32_t count, hipStream_t stream) {
  const unsigned blocks = (count + 63u) / 64u;
  if (ok)
    kem_key_kernel<ID, true><<<dim3(blocks), dim3(64), 0, stream>>>(m, sigma, ok, u, v, key, count);
  else
    kem_key_kernel<ID, false><<<dim3(blocks), dim3(64), 0, stream>>>(m, m, nullptr, u, v, key, count);
  return hipGetLastError();
}

}  // namespace

uint32_t kem_draw_words(int pid) {
  switch (pid) {
    case 1: return KemGeo<1>::NDRAW;
    case 3: return KemGeo<3>::NDRAW;
    default: return KemGeo<5>::NDRAW;
  }
}

uint32_t kem_draw_stride(int pid) {
  switch (pid) {
    case 1: return KemGeo<1>::STRIDE;
    case 3: return KemGeo<3>::STRIDE;
    default: return KemGeo<5>::STRIDE;
  }
}

hipError_t launch_kem_draws(int pid, const uint8_t *m, uint32_t *draws, uint32_t count,
                            hipStream_t stream) {
  switch (pid) {
    case 1: return draws_for<1>(m, draws, count, stream);
    case 3: return draws_for<3>(m, draws, count, stream);
    default: return draws_for<5>(m, draws, count, stream);
  }
}

hipError_t launch_kem_key(int pid, const uint8_t *m, const uint8_t *sigma, const uint32_t *ok,
                          const uint64_t *u, const uint64_t *v, uint8_t *key, uint32_t count,
                          hipStream_t stream) {
  switch (pid) {
    case 1: return key_for<1>(m, sigma, ok, u, v, key, count, stream);
    case 3: return key_for<3>(m, sigma, ok, u, v, key, count, stream);
    default: return key_for<5>(m, sigma, ok, u, v, key, count, stream);
  }
}

// ---- fixed scratch for the allocation-free decapsulation ----------------------
// A file-scope device array: the code object holds one instance per device,
// for the life of the process.  Host code uses only the address that
// hipGetSymbolAddress returns for the current device (the array's name in
// host code is a host-side stand-in, not a device address).
namespace {
__device__ __align__(256) unsigned char scratch[HQC_NOALLOC_SCRATCH_BYTES];

struct ScratchAddr {
  std::mutex mu;
  std::map<int, void *> ptr;  // device -> address of its scratch
};
ScratchAddr g_scratch;
}  // namespace

hipError_t noalloc_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_scratch.mu);
  auto it = g_scratch.ptr.find(dev);
  if (it == g_scratch.ptr.end()) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = g_scratch.ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return hipSuccess;
}

}  // namespace hqc
