// hqc_encrypt.hip -- batched HQC key generation (Alg. 3: s = x + h*y) and
// PKE encryption (Alg. 1: u = r1 + h*r2, v = mG + s*r2 + e truncated to
// n1*n2 bits) for gfx950.  The randomness (h, x, y, r1, r2, e, m) is an
// input; nothing here draws random numbers.  For the KEM, the supports r1,
// r2, e can instead be sampled in the kernel from 32-bit draws (Floyd's
// sampling), and the result compared with a received ciphertext instead of
// stored (the re-encryption check of decapsulation).
//
// One 64-lane wavefront per item (persistent grid).  Dense operands are
// staged as a bit-level doubled copy in LDS and multiplied by the sparse
// operand with the windowed product of Eq. (1) shared with decryption.  The
// sparse addends (x, r1, e) are added as products with the constant
// polynomial 1, so their secret positions never become memory addresses.
// The codeword mG: Reed-Solomon parity by a wavefront-wide LFSR (lane j
// holds register j; GF(2^8) products through the wave-resident log/exp
// tables), then each output dword of the duplicated RM(1,7) code from its
// symbol: a 32-entry pattern table for the low five message bits (read with
// ds_bpermute_b32) and a whole-dword complement for bits 5-7.
#include "hqc_device.h"
#include "hqc_internal_enc.h"

namespace hqc {
namespace {

// log g_j (and g_j != 0) for g(x) = prod_{i=1}^{2d} (x - alpha^i)
struct RsGenTables {
  uint8_t lg[3][64];
  uint8_t nz[3][64];
};

constexpr RsGenTables make_rs_gen_tables() {
  RsGenTables t{};
  uint8_t e[256] = {}, l[256] = {};
  unsigned x = 1;
  for (int i = 0; i < 255; ++i) {
    e[i] = (uint8_t)x;
    l[x] = (uint8_t)i;
    x <<= 1;
    if (x & 0x100u) x ^= 0x11Du;
  }
  const int tds[3] = {30, 32, 58};
  for (int s = 0; s < 3; ++s) {
    uint8_t g[64] = {};
    g[0] = 1;
    for (int i = 1; i <= tds[s]; ++i) {
      // g <- g * (x + alpha^i)
      for (int d = i; d >= 0; --d) {
        uint8_t lo = g[d] ? e[(l[g[d]] + i) % 255] : 0;  // alpha^i * g_d
        uint8_t hi = d > 0 ? g[d - 1] : 0;               // x * g (coefficient d)
        g[d] = (uint8_t)(hi ^ lo);
      }
    }
    for (int j = 0; j < 64; ++j) {
      t.nz[s][j] = (uint8_t)(j < tds[s] && g[j] != 0);
      t.lg[s][j] = g[j] ? l[g[j]] : 0;
    }
  }
  return t;
}

__constant__ RsGenTables kRsGen = make_rs_gen_tables();

template <int ID> constexpr int gen_slot() { return ID == 1 ? 0 : ID == 3 ? 1 : 2; }

// bit i of pattern(v) = parity(v & i) for the low five bits (i = 0 .. 31)
__device__ __forceinline__ uint32_t rm_pattern(uint32_t v) {
  uint32_t p = 0;
  p ^= (v & 1u) ? 0xAAAAAAAAu : 0u;
  p ^= (v & 2u) ? 0xCCCCCCCCu : 0u;
  p ^= (v & 4u) ? 0xF0F0F0F0u : 0u;
  p ^= (v & 8u) ? 0xFF00FF00u : 0u;
  p ^= (v & 16u) ? 0xFFFF0000u : 0u;
  return p;
}

// Stage the dense polynomial a (dwords 0 .. DW of a row) into U2 and make
// the doubled copy.
template <int ID>
__device__ __forceinline__ void stage_dense(const uint64_t *row, uint32_t *u2) {
  using G = Geo<ID>;
  const uint32_t *src = (const uint32_t *)row;
  for (int d = lane_id(); d <= G::DW; d += 64) u2[d] = src[d];
  build_doubled<ID>(u2);
}

template <int NIDX>
__device__ __forceinline__ void load_support(const uint32_t *src, uint32_t (&reg)[(NIDX + 63) / 64]) {
#pragma unroll
  for (int c = 0; c < (NIDX + 63) / 64; ++c) {
    const int idx = 64 * c + lane_id();
    reg[c] = idx < NIDX ? src[idx] : 0u;
  }
}

// Floyd's sampling (Bentley & Floyd 1987, positions reflected): W distinct
// positions in [0, n) from W 32-bit draws a_i.  p_i = i + floor(a_i (n - i)
// / 2^32); then for i = W-1 down to 0, p_i becomes i if a later p_j equals
// it.  Position i is kept in lane i mod 64 of p[i / 64]; the loop length and
// every access are fixed, the replacement is a select.
template <int ID, int W>
__device__ __forceinline__ void floyd(const uint32_t *a, uint32_t (&p)[(W + 63) / 64]) {
  constexpr int NR = (W + 63) / 64;
  constexpr uint32_t n = (uint32_t)Set<ID>::n;
  const int lane = lane_id();
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    const int i = 64 * c + lane;
    const uint32_t ai = a[i < W ? i : 0];
    p[c] = i < W ? (uint32_t)i + __umulhi(ai, n - (uint32_t)i) : 0xFFFFFFFFu;  // never a position
  }
#pragma unroll
  for (int c = NR - 1; c >= 0; --c) {
    const int top = W - 64 * c < 64 ? W - 64 * c : 64;
#pragma unroll 1
    for (int l = top - 1; l >= 0; --l) {
      const int i = 64 * c + l;
      const uint32_t pi = rdlane(p[c], l);
      bool hit = false;
#pragma unroll
      for (int c2 = c; c2 < NR; ++c2) hit |= (64 * c2 + lane > i) && p[c2] == pi;
      const bool dup = __ballot(hit) != 0ull;
      p[c] = (dup && lane == l) ? (uint32_t)i : p[c];
    }
  }
}

// a*(support) + 1*(support2) -> acc (all R dwords of every lane); supports
// held lane-strided in registers
template <int ID, int N1, int N2>
__device__ __forceinline__ void two_products(const uint32_t *u2, const uint32_t *one,
                                             const uint32_t (&i1)[(N1 + 63) / 64],
                                             const uint32_t (&i2)[(N2 + 63) / 64],
                                             uint32_t (&acc)[Geo<ID>::R]) {
  uint32_t s1[(N1 + 63) / 64], s2[(N2 + 63) / 64];
  window_shifts<ID, (N1 + 63) / 64>(i1, s1);
  window_shifts<ID, (N2 + 63) / 64>(i2, s2);
#pragma unroll
  for (int j = 0; j < Geo<ID>::R; ++j) acc[j] = 0;
  product_acc<ID, N1>(u2, s1, acc);
  product_acc<ID, N2>(one, s2, acc);
}

// store a full n-bit polynomial (bits >= n cleared) from the lanes' dwords,
// or (CHECK) return the OR of its differences from the stored row
template <int ID, bool CHECK>
__device__ __forceinline__ uint32_t store_full(uint64_t *row, const uint64_t *cmp,
                                               const uint32_t (&acc)[Geo<ID>::R]) {
  using G = Geo<ID>;
  uint32_t *dst = (uint32_t *)row;
  const uint32_t *src = (const uint32_t *)cmp;
  const int lane = lane_id();
  uint32_t diff = 0;
#pragma unroll
  for (int j = 0; j < G::R; ++j) {
    const int d = lane * G::R + j;
    if (d < 2 * G::U_WORDS) {
      uint32_t val = d < G::DW ? acc[j] : (d == G::DW ? acc[j] & ((1u << G::NB) - 1u) : 0u);
      if constexpr (CHECK)
        diff |= src[d] ^ val;
      else
        dst[d] = val;
    }
  }
  return diff;
}

template <int ID, int MODE>
__device__ __forceinline__ void run_item(const EncArgs &a, uint32_t item, uint32_t *lds,
                                         uint32_t exp4, uint32_t log4, uint32_t pat) {
  using G = Geo<ID>;
  const int lane = lane_id();
  uint32_t *u2 = lds;
  uint32_t *one = lds + G::U2;
  uint8_t *sym = (uint8_t *)(lds + 2 * G::U2);
  uint32_t acc[G::R];
  const size_t nw = (size_t)G::U_WORDS;

  if constexpr (MODE == ENC_KEYGEN) {
    // Alg. 3: s = x + h*y
    constexpr int NR = (G::w + 63) / 64;
    uint32_t iy[NR], ix[NR];
    load_support<G::w>(a.y + (size_t)item * G::w, iy);
    load_support<G::w>(a.x + (size_t)item * G::w, ix);
    stage_dense<ID>(a.h + item * nw, u2);
    two_products<ID, G::w, G::w>(u2, one, iy, ix, acc);
    store_full<ID, false>(a.s_out + item * nw, nullptr, acc);
    wave_sync();
    return;
  } else {
    constexpr int WR = Set<ID>::wr, WE = Set<ID>::we;
    constexpr bool CHECK = MODE == ENC_CHECK;
    uint32_t ir1[(WR + 63) / 64], ir2[(WR + 63) / 64], ie[(WE + 63) / 64];
    if constexpr (MODE == ENC_ARRAYS) {
      load_support<WR>(a.r1 + (size_t)item * WR, ir1);
      load_support<WR>(a.r2 + (size_t)item * WR, ir2);
      load_support<WE>(a.e + (size_t)item * WE, ie);
    } else {
      const uint32_t *dr = a.draws + (size_t)item * a.draw_stride;
      floyd<ID, WR>(dr, ir1);
      floyd<ID, WR>(dr + WR, ir2);
      floyd<ID, WE>(dr + 2 * WR, ie);
    }
    // Alg. 1: u = r1 + h*r2
    stage_dense<ID>(a.h + item * nw, u2);
    two_products<ID, WR, WR>(u2, one, ir2, ir1, acc);
    uint32_t diff = store_full<ID, CHECK>(a.u_out + item * nw, a.u_in + item * nw, acc);

    // Reed-Solomon parity of m: x^{2d} m(x) mod g(x), register j in lane j
    constexpr int TD = G::TD;
    const uint8_t *mrow = a.m + (size_t)item * G::k;
    const uint32_t mlane = lane < G::k ? (uint32_t)mrow[lane] : 0u;  // byte t of m in lane t
    const uint32_t lg = kRsGen.lg[gen_slot<ID>()][lane];
    const uint32_t gnz = kRsGen.nz[gen_slot<ID>()][lane];
    uint32_t reg = 0;
#pragma unroll 1
    for (int t = G::k - 1; t >= 0; --t) {
      const uint32_t mt = rdlane(mlane, t);
      const uint32_t fb = (mt ^ rdlane(reg, TD - 1)) & 0xFFu;
      const uint32_t lfb = tab(log4, fb);
      uint32_t prod = tab(exp4, red255(lfb + lg));
      prod = (fb != 0 && gnz) ? prod : 0u;
      const uint32_t prev = (uint32_t)__builtin_amdgcn_ds_bpermute((lane > 0 ? lane - 1 : 0) << 2,
                                                                  (int)reg);
      reg = lane < TD ? ((lane > 0 ? prev : 0u) ^ prod) : 0u;
    }
    if (lane < TD) sym[lane] = (uint8_t)reg;
    if (lane < G::k) sym[TD + lane] = (uint8_t)mlane;

    // v = mG + s*r2 + e, first n1*n2 bits
    wave_sync();
    stage_dense<ID>(a.s + item * nw, u2);
    two_products<ID, WR, WE>(u2, one, ir2, ie, acc);
    uint32_t *dst = (uint32_t *)(a.v_out + item * (size_t)G::V_WORDS);
    const uint32_t *vin = (const uint32_t *)(a.v_in + item * (size_t)G::V_WORDS);
#pragma unroll
    for (int j = 0; j < G::R; ++j) {
      const int d = lane * G::R + j;
      const int dd = d < G::W32 ? d : 0;
      const int blk = dd / G::BLK, w = (dd % G::BLK) & 3;
      const uint32_t c = sym[blk];
      const uint32_t p = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((c & 31u) << 2), (int)pat);
      const uint32_t flip = ((c >> 7) ^ ((c >> 5) & (uint32_t)w) ^ ((c >> 6) & ((uint32_t)w >> 1))) & 1u;
      const uint32_t word = p ^ (0u - flip);
      if (d < G::W32) {
        if constexpr (CHECK)
          diff |= vin[d] ^ acc[j] ^ word;
        else
          dst[d] = acc[j] ^ word;
      }
    }
    if constexpr (CHECK) {
      const bool same = __ballot(diff != 0u) == 0ull;
      if (lane == 0) a.ok[item] = same ? 1u : 0u;
    }
    wave_sync();
  }
}

template <int MODE, int ID>
__global__ __launch_bounds__(64) void hqc_encrypt_kernel(EncArgs a) {
  extern __shared__ uint32_t lds[];
  using G = Geo<ID>;
  const int lane = lane_id();
  const uint32_t exp4 = kGf.exp4[lane];
  const uint32_t log4 = kGf.log4[lane];
  const uint32_t pat = rm_pattern((uint32_t)lane & 31u);
  // the doubled copy of the constant polynomial 1: bits 0 and n
  uint32_t *one = lds + G::U2;
  for (int d = lane; d < G::U2; d += 64) one[d] = 0;
  wave_sync();
  if (lane == 0) {
    one[0] = 1u;
    one[G::DW] = 1u << G::NB;
  }
  wave_sync();
  for (uint32_t item = blockIdx.x; item < a.count; item += gridDim.x)
    run_item<ID, MODE>(a, item, lds, exp4, log4, pat);
}

template <int ID> size_t enc_lds() {
  using G = Geo<ID>;
  return sizeof(uint32_t) * 2 * G::U2 + ((G::n1 + 63) / 64) * 64;
}

}  // namespace

template <int MODE> const void *enc_ptr(int pid) {
  switch (pid) {
    case 1: return (const void *)&hqc_encrypt_kernel<MODE, 1>;
    case 3: return (const void *)&hqc_encrypt_kernel<MODE, 3>;
    default: return (const void *)&hqc_encrypt_kernel<MODE, 5>;
  }
}

const void *encrypt_kernel_ptr(int mode, int pid) {
  switch (mode) {
    case ENC_KEYGEN: return enc_ptr<ENC_KEYGEN>(pid);
    case ENC_ARRAYS: return enc_ptr<ENC_ARRAYS>(pid);
    case ENC_STREAM: return enc_ptr<ENC_STREAM>(pid);
    default: return enc_ptr<ENC_CHECK>(pid);
  }
}

size_t encrypt_lds_bytes(int pid) {
  switch (pid) {
    case 1: return enc_lds<1>();
    case 3: return enc_lds<3>();
    default: return enc_lds<5>();
  }
}

hipError_t launch_encrypt(int mode, int pid, const EncArgs &a, int grid, hipStream_t stream) {
  EncArgs copy = a;
  void *args[] = {&copy};
  return hipLaunchKernel(encrypt_kernel_ptr(mode, pid), dim3((unsigned)grid), dim3(64), args,
                         encrypt_lds_bytes(pid), stream);
}

}  // namespace hqc
