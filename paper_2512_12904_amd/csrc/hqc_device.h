// hqc_device.h -- device-side pieces shared by the decryption kernels
// (hqc_kernels.hip) and the key-generation / encryption kernels
// (hqc_encrypt.hip): parameter geometry (Table I), GF(2^8) tables, lane
// helpers, the bit-level doubled copy of a dense polynomial in LDS and the
// windowed sparse x dense product of Eq. (1).
#pragma once

#include "hqc_internal.h"

namespace hqc {
namespace {

// ---- parameter sets (Table I) --------------------------------------------
template <int ID> struct Set;
template <> struct Set<1> { static constexpr int n = 17669, n1 = 46, n2 = 384, k = 16, delta = 15, w = 66, wr = 75, we = 75; };
template <> struct Set<3> { static constexpr int n = 35851, n1 = 56, n2 = 640, k = 24, delta = 16, w = 100, wr = 114, we = 114; };
template <> struct Set<5> { static constexpr int n = 57637, n1 = 90, n2 = 640, k = 32, delta = 29, w = 131, wr = 149, we = 149; };

// smallest multiple of 4 bytes >= b whose dword count is odd (so that 64
// lanes reading the same offset of their own rows hit distinct banks)
constexpr int odd_dword_stride(int b) {
  int d = (b + 3) / 4;
  return 4 * (d | 1);
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Kernel shapes of the decryption kernels (SH, a tuning knob; results never
// depend on it): shape 0 for every set, and shape 1 for HQC-1 and HQC-3,
// built for three wavefronts per SIMD instead of two (HQC-3 with the compact
// LDS layout to fit them).  SH 2 is the layout of the decoding kernels'
// shape 0: decoding needs no doubled u, so their LDS holds the received
// words and the symbol table only, and three wavefronts per SIMD fit for
// every set.  Key generation and encryption use shape 0's sizes.
template <int ID, int SH = 0> struct Geo {
  static_assert(SH == 0 || SH == 2 || (SH == 1 && ID != 5), "shape 1 exists for HQC-1 and HQC-3");
  using S = Set<ID>;
  static constexpr int n = S::n, n1 = S::n1, n2 = S::n2, k = S::k, w = S::w;
  static constexpr int MULT = n2 / 128;
  static constexpr int TD = 2 * S::delta;            // number of syndromes
  static constexpr int W32 = n1 * n2 / 32;           // dwords of v and of the product we keep
  static constexpr int R = ((W32 + 63) / 64) | 1;    // product dwords per lane (odd)
  static constexpr int DW = n / 32;                  // dword holding bit n - 1
  static constexpr int NB = n % 32;                  // bits of u in that dword
  static constexpr int U_WORDS = (n + 63) / 64;
  static constexpr int V_WORDS = n1 * n2 / 64;
  static constexpr int BLK = 4 * MULT;               // dwords per RM block
  static constexpr int BSTR = BLK + 1;               // padded LDS row of a block
  static constexpr int U2 = 64 * R + DW + 2;         // doubled-u dwords (covers every window)
  static constexpr int RB = n1 * BSTR;               // received-word dwords
  static constexpr int YREG = (w + 63) / 64;         // VGPRs holding y
  static constexpr int SSTR = odd_dword_stride(n1);  // symbol-table row (bytes)
  // HQC-5 (and HQC-3 in shape 1) runs a tile as sub-tiles of at most 32
  // items (two lanes per Reed-Solomon word) and builds the received word over
  // the doubled u once the product is in registers, so that one wavefront
  // fits in 20 KiB of LDS (eight wavefronts per CU; HQC-3 shape 1: 11 KiB)
  static constexpr bool COMPACT = ID == 5 || (ID == 3 && SH == 1);
  static constexpr int TROWS = COMPACT ? 32 : 64;    // items per (sub-)tile
  static constexpr bool DECODE_ONLY = SH == 2;       // no doubled u in LDS
  static constexpr int RB_OFF = (COMPACT || DECODE_ONLY) ? 0 : U2;  // dword offset of the received word
  // RM blocks are decoded 32 per pass, one per lane pair (matrix cores).
  // HQC-1 keeps the received words of RMG = 2 items and decodes their
  // 2 x 46 = 92 blocks in 3 passes instead of 2 x 2
  static constexpr int RMG = ID == 1 ? 2 : 1;
  static constexpr int WAVES = SH == 0 ? 2 : 3;      // wavefronts per SIMD the kernel is built for
  static constexpr int A_BYTES =
      DECODE_ONLY ? (4 * RMG * RB + 15) / 16 * 16
                  : (4 * (COMPACT ? cmax(U2, RB) : U2 + RMG * RB) + 15) / 16 * 16;
  static constexpr int LDS_BYTES = A_BYTES + TROWS * SSTR;
  // debug dump of one item (byte offsets; the record is a whole number of dwords)
  static constexpr int DBG_SYM = 4 * W32, DBG_S = DBG_SYM + n1, DBG_LAM = DBG_S + TD,
                       DBG_E = DBG_LAM + TD + 1, DBG_BYTES = (DBG_E + k + 3) / 4 * 4;
  static_assert(NB != 0, "n is not a multiple of 32 for any HQC set");
  static_assert(TD + 1 <= 64 && k <= 64, "lane-level sizes");
  static_assert(n1 * n2 % 64 == 0, "v is a whole number of words");
  static_assert(64 * R >= W32, "lanes cover the product");
  static_assert(TD + k == n1 && n1 < 255, "message positions");
  static_assert(LDS_BYTES * 4 * WAVES <= 160 * 1024, "LDS of the wavefronts per CU");
};

// ---- LDS and row index expressions -----------------------------------------
// The index arithmetic of the kernels' LDS and row accesses, for geometry G.
// The kernels compute their addresses with these functions, and a host-side
// check (tests) evaluates the same functions over every lane, shift, tile
// row and pass against the LDS and buffer sizes.  Offsets are in dwords
// from the start of the dynamic LDS, except the symbol tables (bytes).
// The persistent grid's tile schedule: workgroup `block` of `grid` takes
// tiles block, block + grid, block + 2 grid, ...; its first tile at or after
// a segment's first tile `first`.
__host__ __device__ constexpr uint32_t first_unit(uint32_t block, uint32_t grid, uint32_t first) {
  return block >= first ? block : block + (first - block + grid - 1) / grid * grid;
}

template <class G> struct Layout {
  static constexpr int BPP = 32;  // RM blocks per pass (one per lane pair)
  // decryption: received-word slot q starts at rb(q); dword d of a word sits
  // at rb(q) + row(d) (one RM block per padded row of BSTR dwords)
  static __host__ __device__ constexpr int rb(int q) { return G::RB_OFF + q * G::RB; }
  static __host__ __device__ constexpr int row(int d) { return d + d / G::BLK; }
  // first dword of block b of slot q
  static __host__ __device__ constexpr int block(int q, int b) { return rb(q) + b * G::BSTR; }
  // dword j (0 .. R) of lane l's product window for the shift sh (doubled copy)
  static __host__ __device__ constexpr int window(int lane, uint32_t sh, int j) {
    return lane * G::R + (int)(sh >> 5) + j;
  }
  // output dword j (0 .. R - 1) of lane l's product
  static __host__ __device__ constexpr int out(int lane, int j) { return lane * G::R + j; }
  // decryption: byte b of row r of the tile's symbol table
  static __host__ __device__ constexpr int sym(int r, int b) { return G::A_BYTES + r * G::SSTR + b; }
  // RM pass p of a group: the flat block index lane takes (q n1 + b for
  // block b of slot q), before clamping to the blocks received
  static __host__ __device__ constexpr int pass_flat(int p, int lane) {
    return BPP * p + (lane & 31);
  }
  static __host__ __device__ constexpr int pass_clamp(int fl, int avail) {
    return fl < avail ? fl : avail - 1;
  }
  // key generation / encryption: byte b of the symbol table after the
  // doubled copy (the output staging buffer starts at dword 0)
  static __host__ __device__ constexpr int enc_sym(int b) { return 4 * G::U2 + b; }
  static constexpr int ENC_LDS_BYTES = 4 * G::U2 + (G::n1 + 63) / 64 * 64;
};

// ---- GF(2^8) tables, x^8 + x^4 + x^3 + x^2 + 1, alpha = x ------------------
// A 256-byte table is held in lanes 0 .. 31, 8 bytes per lane (lo: bytes
// 8l .. 8l+3, hi: 8l+4 .. 8l+7; lanes 32 .. 63 hold a copy).  A lookup
// reads source lane idx / 8 of both registers through the LDS crossbar
// (ds_bpermute_b32): every source lane is below 32, so two lanes reading
// different entries never meet in one bank and the lookup's timing does not
// depend on the secret index.
struct GfTables {
  uint32_t exp_lo[32], exp_hi[32];  // exp[i] = alpha^i, exp[255] = exp[0] = 1
  uint32_t log_lo[32], log_hi[32];  // log[0] = 0 (callers mark zero)
};

constexpr GfTables make_gf_tables() {
  GfTables t{};
  uint8_t e[256] = {}, l[256] = {};
  unsigned x = 1;
  for (int i = 0; i < 255; ++i) {
    e[i] = (uint8_t)x;
    l[x] = (uint8_t)i;
    x <<= 1;
    if (x & 0x100u) x ^= 0x11Du;
  }
  e[255] = 1;
  auto word = [](const uint8_t *b) {
    return (uint32_t)b[0] | (uint32_t)b[1] << 8 | (uint32_t)b[2] << 16 | (uint32_t)b[3] << 24;
  };
  for (int i = 0; i < 32; ++i) {
    t.exp_lo[i] = word(e + 8 * i);
    t.exp_hi[i] = word(e + 8 * i + 4);
    t.log_lo[i] = word(l + 8 * i);
    t.log_hi[i] = word(l + 8 * i + 4);
  }
  return t;
}

__constant__ GfTables kGf = make_gf_tables();

struct GfTab {
  uint32_t lo, hi;
};

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// A log value >= ZL stands for the log of zero; sums of two logs and one
// reduction step keep it >= 512.
constexpr uint32_t ZL = 0x400;

__device__ __forceinline__ int lane_id() { return (int)threadIdx.x; }

// The workgroup is one wavefront and a wavefront's LDS operations complete in
// issue order, so ordering LDS traffic between lanes needs no s_barrier; the
// wavefront-scope fences only stop the compiler from moving memory
// operations across this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Byte idx (0..255) of a table held as above.  Must run with all 64 lanes
// active.  width 8 returns the byte, width 0 returns 0.
__device__ __forceinline__ uint32_t tab(GfTab t, uint32_t idx, uint32_t width = 8) {
  const int src = (int)((idx >> 1) & 0x7Cu);  // byte address of lane (idx / 8) mod 32
  const uint32_t a = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)t.lo);
  const uint32_t b = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)t.hi);
  return __builtin_amdgcn_ubfe((idx & 4u) ? b : a, (idx & 3u) << 3, width);
}

__device__ __forceinline__ GfTab gf_exp_tab() {
  const int l = lane_id() & 31;
  return {kGf.exp_lo[l], kGf.exp_hi[l]};
}
__device__ __forceinline__ GfTab gf_log_tab() {
  const int l = lane_id() & 31;
  return {kGf.log_lo[l], kGf.log_hi[l]};
}

// s mod 255 for s in [0, 509] (as an exp index in [0, 254])
__device__ __forceinline__ uint32_t red255(uint32_t s) {
  uint32_t t = s - 255u;
  return t < s ? t : s;  // unsigned: t wraps above s when s < 255
}

// log with zero marked: log(x), or ZL (+ log[0]) when x == 0
__device__ __forceinline__ uint32_t logz(GfTab log4, uint32_t x) {
  return tab(log4, x) | (x == 0 ? ZL : 0u);
}

// alpha^s for a sum of logs s (0 when s carries a zero mark)
__device__ __forceinline__ uint32_t expz(GfTab exp4, uint32_t s) {
  uint32_t v = tab(exp4, red255(s) & 0xFFu);
  return s < 512u ? v : 0u;
}

// three-input bitwise functions (v_bitop3_b32, truth table over the inputs)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}

__device__ __forceinline__ uint32_t rdlane(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// v_permlane32_swap_b32 on two copies of x: .lo is lane (l mod 32)'s x and
// .hi is lane (l mod 32) + 32's x, in every lane l
struct Halves {
  uint32_t lo, hi;
};
__device__ __forceinline__ Halves halves(uint32_t x) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return {r[0], r[1]};
}


// ---- S0 / S1 building blocks -------------------------------------------------

// U2[t] = a[t mod n] for t < 2n (zero above): U2[0 .. DW] must already hold
// dwords 0 .. DW of a (dword DW raw; bits >= n there are ignored).  Called by
// all 64 lanes.
template <int ID>
__device__ __forceinline__ void build_doubled(uint32_t *u2) {
  using G = Geo<ID>;
  const int lane = lane_id();
  wave_sync();
  const uint32_t udw = u2[G::DW] & ((1u << G::NB) - 1u);
  const uint32_t u0 = u2[0];
  wave_sync();
  for (int D = G::DW + lane; D < G::U2; D += 64) {
    const int i = D - G::DW;  // >= 0
    uint32_t val;
    if (i == 0) {
      val = udw | (u0 << G::NB);
    } else {
      const int ih = i < G::DW ? i : G::DW - 1, il = i - 1 < G::DW ? i - 1 : G::DW - 1;
      uint32_t hi = i < G::DW ? u2[ih] : (i == G::DW ? udw : 0u);
      uint32_t lo = i - 1 < G::DW ? u2[il] : (i - 1 == G::DW ? udw : 0u);
      val = __builtin_amdgcn_alignbit(hi, lo, 32 - G::NB);
    }
    u2[D] = val;
  }
  wave_sync();
}

// The same doubled copy written from registers: ur[c] holds dword lane + 64c
// of a (c < NR, dwords 0 .. DW).  U2[DW + i] takes the bits of dwords i - 1
// and i of a, the previous dword coming from the next lower lane through a
// wave-wide DPP shift (lane 0 takes lane 63 of the previous register), so no
// LDS read is needed.  Called by all 64 lanes; the caller orders these LDS
// writes before the first read.
template <int ID, int NR>
__device__ __forceinline__ void build_doubled_regs(uint32_t *u2, const uint32_t (&ur)[NR]) {
  using G = Geo<ID>;
  const int lane = lane_id();
  constexpr int NC = (G::U2 - G::DW + 63) / 64;
  static_assert(G::DW / 64 < NR, "the top dword is held");
  const uint32_t udw = rdlane(ur[G::DW / 64], G::DW % 64) & ((1u << G::NB) - 1u);
  uint32_t carry = udw << (32 - G::NB);  // makes U2[DW] = udw | a0 << NB
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int j = lane + 64 * c;
    uint32_t hi = 0u;
    if (c < NR) hi = j < G::DW ? ur[c < NR ? c : 0] : (j == G::DW ? udw : 0u);
    // wave_shr:1 -- lane l reads lane l - 1, lane 0 keeps carry
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)carry, (int)hi, 0x138, 0xF, 0xF, false);
    const int D = G::DW + j;
    if (D < G::U2) u2[D] = __builtin_amdgcn_alignbit(hi, lo, 32 - G::NB);
    carry = rdlane(hi, 63);
  }
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    const int d = lane + 64 * c;
    if (d < G::DW) u2[d] = ur[c];
  }
}

// shreg for NIDX support indices held lane-strided in idx[] (index 64c + l in
// lane l of idx[c]): sh = n - (index mod n) in [1, n]
template <int ID, int NREG>
__device__ __forceinline__ void window_shifts(const uint32_t (&idx)[NREG], uint32_t (&sh)[NREG]) {
  using G = Geo<ID>;
#pragma unroll
  for (int c = 0; c < NREG; ++c) sh[c] = (uint32_t)G::n - idx[c] % (uint32_t)G::n;
}

// NP pairs of shifts, from packed dwords p .. p + NP - 1 of pk (two 16-bit
// shifts a dword): their 2 NP windows are loaded together, then each pair is
// combined with a three-way XOR
template <int ID, int NP>
__device__ __forceinline__ void product_pairs(const uint32_t *u2, uint32_t pk, int p, int lane,
                                              uint32_t (&acc)[Geo<ID>::R]) {
  using G = Geo<ID>;
  using L = Layout<G>;
  uint32_t win[2 * NP][G::R + 1], shs[2 * NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const uint32_t w = rdlane(pk, p + q);
    shs[2 * q] = w & 0xFFFFu;
    shs[2 * q + 1] = w >> 16;
  }
#pragma unroll
  for (int q = 0; q < 2 * NP; ++q)
#pragma unroll
    for (int j = 0; j <= G::R; ++j) win[q][j] = u2[L::window(lane, shs[q], j)];
#pragma unroll
  for (int q = 0; q < 2 * NP; q += 2)
#pragma unroll
    for (int j = 0; j < G::R; ++j)
      acc[j] = xor3(acc[j], __builtin_amdgcn_alignbit(win[q][j + 1], win[q][j], shs[q]),
                    __builtin_amdgcn_alignbit(win[q + 1][j + 1], win[q + 1][j], shs[q + 1]));
}

// acc[j] ^= bits [32 (lane R + j) + sh_k, +32) of U2 for the first NIDX
// shifts: lane l's R output dwords of (sum_k X^{index_k}) * a, restricted to
// the dwords below 64 R.  The shifts of a register's cnt indices are first
// packed two to a dword (lane l < cnt / 2 holds those of lanes l and
// l + ceil(cnt / 2); every shift is at most n < 2^16), so one lane read
// serves two indices; the windows of U indices are loaded together, then
// combined two at a time with a three-way XOR.  The XOR sum does not depend
// on the order the indices are taken in.
template <int ID, int NIDX>
__device__ __forceinline__ void product_acc(const uint32_t *u2,
                                            const uint32_t (&shreg)[(NIDX + 63) / 64],
                                            uint32_t (&acc)[Geo<ID>::R]) {
  using G = Geo<ID>;
  static_assert(G::n < 65536, "shifts are packed as 16-bit halves");
  constexpr int NREG = (NIDX + 63) / 64;
  using L = Layout<G>;
  const int lane = lane_id();
  constexpr int U = G::R <= 10 ? 4 : 2;
#pragma unroll
  for (int c = 0; c < NREG; ++c) {
    const int cnt = (NIDX - 64 * c) < 64 ? (NIDX - 64 * c) : 64;
    const int half = (cnt + 1) / 2;
    uint32_t hi;
    if (half == 32) {
      hi = halves(shreg[c]).hi;
    } else {
      // lane (l + half) mod 64's shift; lanes past the register's indices
      // read values that are never used
      hi = (uint32_t)__builtin_amdgcn_ds_bpermute((lane + half) << 2, (int)shreg[c]);
    }
    const uint32_t pk = shreg[c] | hi << 16;
    const int np = cnt / 2;
    int p = 0;
    for (; p + U / 2 <= np; p += U / 2) product_pairs<ID, U / 2>(u2, pk, p, lane, acc);
    if constexpr (U / 2 > 1)
      for (; p < np; ++p) product_pairs<ID, 1>(u2, pk, p, lane, acc);
    if (cnt & 1) {
      // the odd index: lane np's low half
      uint32_t win[G::R + 1];
      const uint32_t sh = rdlane(pk, np) & 0xFFFFu;
#pragma unroll
      for (int j = 0; j <= G::R; ++j) win[j] = u2[L::window(lane, sh, j)];
#pragma unroll
      for (int j = 0; j < G::R; ++j) acc[j] ^= __builtin_amdgcn_alignbit(win[j + 1], win[j], sh);
    }
  }
}

}  // namespace
}  // namespace hqc
