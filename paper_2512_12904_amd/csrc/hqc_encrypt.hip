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
// sparse addends (x, r1, e) are added one bit per index, either into the
// product registers (the owning lane selects it; the register is addressed
// with the VGPR index mode) or into the LDS staging buffer with one atomic
// XOR per index issued by that index's lane alone; either way the
// instructions and their timing do not depend on the secret positions.  The
// result goes through the LDS buffer to coalesced stores (or is compared
// with a received ciphertext).  Rows of h and s are loaded an item ahead.
// The codeword mG: Reed-Solomon parity as a GF(2)-linear map of the message
// bits (lane j sums its parity byte over rows selected by the bits; no
// table index depends on m), then each output dword of the duplicated
// RM(1,7) code from its
// symbol: a 32-entry pattern table for the low five message bits (read with
// ds_bpermute_b32) and a whole-dword complement for bits 5-7.
#include "hqc_device.h"
#include "hqc_internal_enc.h"

namespace hqc {
namespace {

// Reed-Solomon parity as a GF(2)-linear map of the message bits: the
// parity of m is x^(2d) m(x) mod g(x), g(x) = prod_{i=1}^{2d} (x - alpha^i),
// which is the XOR over the set bits b of the bytes m_t of the parity of the
// one-bit message alpha^b x^t.  Row (t, b) is that parity, 2d bytes; byte
// j of it belongs to lane j.  The table is laid out [set][t][b / 4][lane],
// byte b mod 4 of each dword, so that a lane reads its bytes of four rows
// with one dword load and a wavefront's load is one contiguous block.
template <int ID> struct RsRows {
  static constexpr int K = Set<ID>::k;
  uint32_t w[2 * K][64];
};

template <int ID> constexpr RsRows<ID> make_rs_rows() {
  constexpr int TD = 2 * Set<ID>::delta, K = Set<ID>::k;
  RsRows<ID> t{};
  uint8_t e[256] = {}, l[256] = {};
  unsigned x = 1;
  for (int i = 0; i < 255; ++i) {
    e[i] = (uint8_t)x;
    l[x] = (uint8_t)i;
    x <<= 1;
    if (x & 0x100u) x ^= 0x11Du;
  }
  auto mul = [&](uint8_t a, uint8_t b2) -> uint8_t {
    return (a && b2) ? e[(l[a] + l[b2]) % 255] : 0;
  };
  uint8_t g[64] = {};  // g(x), monic of degree TD
  g[0] = 1;
  for (int i = 1; i <= TD; ++i)
    for (int d = i; d >= 0; --d) g[d] = (uint8_t)((d > 0 ? g[d - 1] : 0) ^ mul(g[d], e[i % 255]));
  for (int tt = 0; tt < K; ++tt)
    for (int b = 0; b < 8; ++b) {
      // remainder of alpha^b x^(TD + tt) divided by g: long division
      uint8_t r[64 + 32] = {};
      r[TD + tt] = (uint8_t)(1u << b);
      for (int d = TD + tt; d >= TD; --d) {
        const uint8_t c = r[d];
        if (!c) continue;
        for (int j = 0; j <= TD; ++j) r[d - TD + j] ^= mul(c, g[j]);
      }
      for (int j = 0; j < TD; ++j) t.w[2 * tt + b / 4][j] |= (uint32_t)r[j] << (8 * (b % 4));
    }
  return t;
}

__constant__ RsRows<1> kRsRows1 = make_rs_rows<1>();
__constant__ RsRows<3> kRsRows3 = make_rs_rows<3>();
__constant__ RsRows<5> kRsRows5 = make_rs_rows<5>();
template <int ID> __device__ __forceinline__ const RsRows<ID> &rs_rows() {
  if constexpr (ID == 1) return kRsRows1;
  else if constexpr (ID == 3) return kRsRows3;
  else return kRsRows5;
}

// four bits of a byte (bits 4h .. 4h + 3) as byte masks 0x00 / 0xFF
__device__ __forceinline__ uint32_t nibble_masks(uint32_t m, int h) {
  const uint32_t x = (m >> (4 * h)) & 0xFu;
  return ((x * 0x00204081u) & 0x01010101u) * 0xFFu;
}

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

// The RS codeword of m into sym[0 .. n1): parity x^(2d) m(x) mod g(x) at
// symbols 0 .. 2d - 1 (lane j < 2d sums its bytes of the rows of the set
// message bits, four bits per dword), message byte t at symbol 2d + t.
// mlane: byte t of m in lane t.  All 64 lanes take part.
template <int ID>
__device__ __forceinline__ void rs_codeword(uint32_t mlane, uint8_t *sym) {
  using G = Geo<ID>;
  const int lane = lane_id();
  const auto &rows = rs_rows<ID>();
  uint32_t racc = 0;
#pragma unroll 4
  for (int t = 0; t < G::k; ++t) {
    const uint32_t mt = rdlane(mlane, t);
    // truth table 0x6C: S1 ^ (S0 & S2)
    racc = __builtin_amdgcn_bitop3_b32(rows.w[2 * t][lane], racc, nibble_masks(mt, 0), 0x6C);
    racc = __builtin_amdgcn_bitop3_b32(rows.w[2 * t + 1][lane], racc, nibble_masks(mt, 1), 0x6C);
  }
  racc ^= racc >> 16;
  const uint32_t reg = (racc ^ (racc >> 8)) & 0xFFu;
  if (lane < G::TD) sym[lane] = (uint8_t)reg;
  if (lane < G::k) sym[G::TD + lane] = (uint8_t)mlane;
}

// dword w (0 .. 3) of the RM(1,7) codeword of symbol c: pattern(c & 31)
// from the lane holding it (pat = rm_pattern(lane & 31); all 64 lanes take
// part), complemented by bit 7 of c and by bits 5, 6 of c where bits 0, 1 of
// w are set
__device__ __forceinline__ uint32_t rm_dword(uint32_t c, uint32_t w, uint32_t pat) {
  const uint32_t p = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((c & 31u) << 2), (int)pat);
  const uint32_t flip = ((c >> 7) ^ ((c >> 5) & w) ^ ((c >> 6) & (w >> 1))) & 1u;
  return p ^ (0u - flip);
}

// registers of one dense row (dwords 0 .. DW, lane-strided)
template <int ID> constexpr int kDenseRegs = (Geo<ID>::DW + 1 + 63) / 64;

// issue the loads of a dense row (dwords 0 .. DW) into registers
template <int ID>
__device__ __forceinline__ void load_dense(const uint64_t *row, uint32_t (&r)[kDenseRegs<ID>]) {
  using G = Geo<ID>;
  const uint32_t *src = (const uint32_t *)row;
#pragma unroll
  for (int c = 0; c < kDenseRegs<ID>; ++c) {
    const int d = lane_id() + 64 * c;
    r[c] = src[d <= G::DW ? d : G::DW];
  }
}

template <int NIDX>
__device__ __forceinline__ void load_support(const uint32_t *src, uint32_t (&reg)[(NIDX + 63) / 64]) {
#pragma unroll
  for (int c = 0; c < (NIDX + 63) / 64; ++c) {
    const int idx = 64 * c + lane_id();
    reg[c] = idx < NIDX ? src[idx] : 0u;
  }
}

// the 3 W draws of one item (r1, r2, e in turn), draw i of vector v in lane
// i mod 64 of p[v][i / 64]
template <int W>
__device__ __forceinline__ void load_draws(const uint32_t *a, uint32_t (&p)[3][(W + 63) / 64]) {
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int c = 0; c < (W + 63) / 64; ++c) {
      const int i = 64 * c + lane_id();
      p[v][c] = a[v * W + (i < W ? i : 0)];
    }
}

// Floyd's sampling (Bentley & Floyd 1987, positions reflected): W distinct
// positions in [0, n) from W 32-bit draws a_i.  p_i = i + floor(a_i (n - i)
// / 2^32); then for i = W-1 down to 0, p_i becomes i if it equals the final
// value of a later p_j.  The three vectors of one encryption (r1, r2, e:
// wr = we in every set) are sampled together.  Position i of vector v is in
// lane i mod 64 of p[v][i / 64].
//
// The steps run over j instead of i: once the final value of p_j is known
// (p_j, or j if p_j was replaced), one ballot marks every i < j whose
// original p_i equals it.  Every i < j is marked by the time j = i + 1 is
// done, so the mark of j is final when j's step starts; the replacement is
// one select per register at the end.  The marks live in 64-bit lane
// masks; a step reads the final value of p_j through a select that takes
// the mask as its lane condition, so the compares of a step do not wait on
// each other and no scalar bit test sits in the chain.  The loop length and
// every access are fixed.
// p holds the draws (load_draws) on entry and the positions on return
template <int ID, int W>
__device__ __forceinline__ void floyd3(uint32_t (&p)[3][(W + 63) / 64]) {
  constexpr int NR = (W + 63) / 64;
  constexpr uint32_t n = (uint32_t)Set<ID>::n;
  const int lane = lane_id();
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const int i = 64 * c + lane;
      p[v][c] = i < W ? (uint32_t)i + __umulhi(p[v][c], n - (uint32_t)i) : 0xFFFFFFFFu;  // never a position
    }
  uint64_t dup[3][NR];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int c = 0; c < NR; ++c) dup[v][c] = 0;
#pragma unroll
  for (int cj = NR - 1; cj >= 0; --cj) {
    const int top = W - 64 * cj < 64 ? W - 64 * cj : 64;
#pragma unroll 4
    for (int lj = top - 1; lj >= 1 - (cj > 0 ? 1 : 0); --lj) {  // j = 64 cj + lj
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        // final value of p_j: j if marked, else p_j (a per-lane select with
        // the mark mask as the lane condition, then one lane read: no
        // scalar bit test in the chain)
        const uint32_t fv =
            __builtin_amdgcn_inverse_ballot_w64(dup[v][cj]) ? (uint32_t)(64 * cj + lane) : p[v][cj];
        const uint32_t fin = rdlane(fv, lj);
#pragma unroll
        for (int c = 0; c <= cj; ++c) {
          const uint64_t below = c < cj ? ~0ull : ((1ull << lj) - 1ull);  // i < j
          dup[v][c] |= __ballot(p[v][c] == fin) & below;
        }
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int c = 0; c < NR; ++c)
      p[v][c] = __builtin_amdgcn_inverse_ballot_w64(dup[v][c]) ? (uint32_t)(64 * c + lane) : p[v][c];
}

// product_acc with the windows of the next group of U indices loaded while
// the current group is combined (two register sets of windows): the LDS
// latency of a group overlaps the previous group's funnel shifts.  The
// shifts are packed as in product_acc; slot 2p and 2p + 1 of a register are
// the two halves of packed dword p (slot cnt - 1 of an odd count: the low
// half alone), and a group of U slots starts at an even slot.
template <int ID, int NIDX>
__device__ __forceinline__ void product_acc_pipelined(const uint32_t *u2,
                                                      const uint32_t (&shreg)[(NIDX + 63) / 64],
                                                      uint32_t (&acc)[Geo<ID>::R]) {
  using G = Geo<ID>;
  static_assert(G::n < 65536, "shifts are packed as 16-bit halves");
  constexpr int NREG = (NIDX + 63) / 64;
  using L = Layout<G>;
  const int lane = lane_id();
  constexpr int U = G::R <= 10 ? 4 : 2;
  static_assert(U % 2 == 0, "groups of whole pairs");
  auto slot = [&](uint32_t pk, int k) {
    const uint32_t w = rdlane(pk, k >> 1);
    return (k & 1) ? w >> 16 : w & 0xFFFFu;
  };
  auto load = [&](uint32_t (&win)[U][G::R + 1], uint32_t (&shs)[U], uint32_t pk, int k0) {
#pragma unroll
    for (int q = 0; q < U; q += 2) {
      const uint32_t w = rdlane(pk, (k0 + q) >> 1);
      shs[q] = w & 0xFFFFu;
      shs[q + 1] = w >> 16;
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int j = 0; j <= G::R; ++j) win[q][j] = u2[L::window(lane, shs[q], j)];
  };
  auto combine = [&](const uint32_t (&win)[U][G::R + 1], const uint32_t (&shs)[U]) {
#pragma unroll
    for (int q = 0; q < U; q += 2)
#pragma unroll
      for (int j = 0; j < G::R; ++j)
        acc[j] = xor3(acc[j], __builtin_amdgcn_alignbit(win[q][j + 1], win[q][j], shs[q]),
                      __builtin_amdgcn_alignbit(win[q + 1][j + 1], win[q + 1][j], shs[q + 1]));
  };
#pragma unroll
  for (int c = 0; c < NREG; ++c) {
    const int cnt = (NIDX - 64 * c) < 64 ? (NIDX - 64 * c) : 64;
    const int half = (cnt + 1) / 2;
    const uint32_t hi = half == 32
                            ? halves(shreg[c]).hi
                            : (uint32_t)__builtin_amdgcn_ds_bpermute((lane + half) << 2, (int)shreg[c]);
    const uint32_t pk = shreg[c] | hi << 16;
    uint32_t wa[U][G::R + 1], wb[U][G::R + 1], sa[U], sb[U];
    int kk = 0;
    if (cnt >= U) load(wa, sa, pk, 0);
    // invariant at the top: wa holds group kk when kk + U <= cnt
    for (; kk + 2 * U <= cnt; kk += 2 * U) {
      load(wb, sb, pk, kk + U);
      combine(wa, sa);
      if (kk + 3 * U <= cnt) load(wa, sa, pk, kk + 2 * U);
      combine(wb, sb);
    }
    if (kk + U <= cnt) {
      combine(wa, sa);
      kk += U;
    }
    for (; kk < cnt; ++kk) {
      uint32_t win[G::R + 1];
      const uint32_t sh = slot(pk, kk);
#pragma unroll
      for (int j = 0; j <= G::R; ++j) win[j] = u2[L::window(lane, sh, j)];
#pragma unroll
      for (int j = 0; j < G::R; ++j) acc[j] ^= __builtin_amdgcn_alignbit(win[j + 1], win[j], sh);
    }
  }
}

// acc = the lane's R dwords of a * (sum over the support of X^index)
template <int ID, int N, bool PIPE = false>
__device__ __forceinline__ void sparse_product(const uint32_t *u2,
                                               const uint32_t (&idx)[(N + 63) / 64],
                                               uint32_t (&acc)[Geo<ID>::R]) {
  uint32_t sh[(N + 63) / 64];
  window_shifts<ID, (N + 63) / 64>(idx, sh);
#pragma unroll
  for (int j = 0; j < Geo<ID>::R; ++j) acc[j] = 0;
  if constexpr (PIPE) product_acc_pipelined<ID, N>(u2, sh, acc);
  else product_acc<ID, N>(u2, sh, acc);
}

// acc ^= the lane's R dwords of sum over the support of X^(index mod n),
// indices >= limit dropped (they add 0 to dword 0).  Lane l holds output
// dwords l R .. l R + R - 1, so index q touches dword q / 32 of lane
// (q / 32) / R, register (q / 32) mod R.  Per index, every lane selects the
// bit (or 0) by comparing its lane number, and the register is addressed
// with the VGPR index mode: no branch, no memory access, the same
// instructions whatever the index.  This replaces a product with the
// constant polynomial 1.
template <int ID, int W>
__device__ __forceinline__ void sparse_xor(uint32_t (&acc)[Geo<ID>::R],
                                           const uint32_t (&p)[(W + 63) / 64], uint32_t limit) {
  using G = Geo<ID>;
  constexpr int NR = (W + 63) / 64;
  const uint32_t lane = (uint32_t)lane_id();
  uint32_t ad[NR], bt[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    const uint32_t q = p[c] % (uint32_t)Set<ID>::n;
    const bool in = q < limit;
    ad[c] = in ? q >> 5 : 0u;
    bt[c] = in ? 1u << (q & 31u) : 0u;
  }
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    const int cnt = W - 64 * c < 64 ? W - 64 * c : 64;
#pragma unroll 4
    for (int l = 0; l < cnt; ++l) {
      const uint32_t a = rdlane(ad[c], l), b = rdlane(bt[c], l);
      const uint32_t owner = a / (uint32_t)G::R, slot = a - owner * (uint32_t)G::R;
      acc[slot] ^= lane == owner ? b : 0u;
    }
  }
}

// buf[q / 32] ^= 1 << (q mod 32) for every index q (taken mod n) of the
// support below limit; indices >= limit are dropped (they XOR 0 into dword
// 0).  Index 64c + l sits in lane l of p[c]; the lanes take turns, one LDS
// atomic XOR each with that lane alone active, so no instruction has two
// lanes that could meet in a bank: the same instructions take the same
// time whatever the positions.  The caller orders the result before reads
// with wave_sync.
template <int ID, int W>
__device__ __forceinline__ void lds_sparse_xor(uint32_t *buf, const uint32_t (&p)[(W + 63) / 64],
                                               uint32_t limit) {
  constexpr int NR = (W + 63) / 64;
  const int lane = lane_id();
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    const uint32_t q = p[c] % (uint32_t)Set<ID>::n;
    const bool in = q < limit;
    uint32_t *const dst = buf + (in ? q >> 5 : 0u);
    const uint32_t bit = in ? 1u << (q & 31u) : 0u;
    const int cnt = W - 64 * c < 64 ? W - 64 * c : 64;
#pragma unroll 8
    for (int l = 0; l < cnt; ++l)
      if (lane == l) __hip_atomic_fetch_xor(dst, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  }
  __builtin_amdgcn_sched_barrier(0);
}

// the lane's R product dwords into buf (bits >= n of the last dword cleared)
template <int ID>
__device__ __forceinline__ void put_full(uint32_t *buf, const uint32_t (&acc)[Geo<ID>::R]) {
  using G = Geo<ID>;
  const int lane = lane_id();
#pragma unroll
  for (int j = 0; j < G::R; ++j) {
    const int d = Layout<G>::out(lane, j);
    if (d <= G::DW) buf[d] = d < G::DW ? acc[j] : acc[j] & ((1u << G::NB) - 1u);
  }
}

// the first ndw dwords of buf to a row (lane-strided, coalesced; dwords
// ndw .. nout - 1 zero)
__device__ __forceinline__ void emit(const uint32_t *buf, int ndw, int nout, uint64_t *row) {
  uint32_t *dst = (uint32_t *)row;
  for (int d = lane_id(); d < nout; d += 64) dst[d] = d < ndw ? buf[d] : 0u;
}

// the first nout dwords of a row into registers (lane-strided), issued
// early so that their latency passes while the product runs
template <int NOUT>
__device__ __forceinline__ void load_row(const uint64_t *row, uint32_t (&r)[(NOUT + 63) / 64]) {
  const uint32_t *src = (const uint32_t *)row;
#pragma unroll
  for (int c = 0; c < (NOUT + 63) / 64; ++c) {
    const int d = lane_id() + 64 * c;
    r[c] = d < NOUT ? src[d] : 0u;
  }
}

// OR of the differences between the first ndw dwords of buf (zero above)
// and the row held by load_row
template <int NOUT>
__device__ __forceinline__ uint32_t compare_row(const uint32_t *buf, int ndw,
                                                const uint32_t (&r)[(NOUT + 63) / 64]) {
  uint32_t diff = 0;
#pragma unroll
  for (int c = 0; c < (NOUT + 63) / 64; ++c) {
    const int d = lane_id() + 64 * c;
    if (d < NOUT) diff |= r[c] ^ (d < ndw ? buf[d] : 0u);
  }
  return diff;
}

// Per-set shape of the encryption kernels, chosen by timing: waves per SIMD
// (the register budget; sampled_waves for the kernels that sample the
// supports from draws: encapsulation and the re-encryption check;
// keygen_waves for key generation, whose product h*y loads the next group
// of windows while the current one is combined when keygen_pipelined --
// HQC-3 and HQC-5, 6 % faster; encryption keeps two rows live and has no
// registers for a second set of windows), whether
// h and s are loaded an item ahead in encryption (pipe; two more rows of
// registers) and h in key generation (keygen_pipe), whether the check
// loads the received u and v before the products that precede their
// comparison (two more rows; for HQC-3 that would cost a wavefront per
// SIMD), and whether the sparse additions r1 and e go into the product
// registers (VGPR index mode, about eight instructions per index) or into
// the LDS staging buffer (one single-lane atomic XOR each).
template <int ID> struct EncShape;
template <> struct EncShape<1> {
  static constexpr int waves = 4, sampled_waves = 5, keygen_waves = 4;
  static constexpr bool keygen_pipelined = false;
  static constexpr bool pipe = true, keygen_pipe = false, check_ahead = true, reg_xor = true;
};
template <> struct EncShape<3> {
  static constexpr int waves = 4, sampled_waves = 4, keygen_waves = 3;
  static constexpr bool keygen_pipelined = true;
  static constexpr bool pipe = true, keygen_pipe = true, check_ahead = false, reg_xor = false;
};
template <> struct EncShape<5> {
  static constexpr int waves = 1, sampled_waves = 1, keygen_waves = 2;
  static constexpr bool keygen_pipelined = true;
  static constexpr bool pipe = true, keygen_pipe = true, check_ahead = true, reg_xor = false;
};

template <int ID, int MODE>
__device__ __forceinline__ void run_item(const EncArgs &a, uint32_t item, uint32_t next,
                                         uint32_t *lds, uint32_t pat,
                                         uint32_t (&hr)[kDenseRegs<ID>]) {
  using G = Geo<ID>;
  const int lane = lane_id();
  // the output staging buffer takes the place of the doubled copy once the
  // product has read it (a wave_sync orders the two)
  uint32_t *u2 = lds;
  uint32_t *buf = lds;
  uint8_t *sym = (uint8_t *)lds + Layout<G>::enc_sym(0);
  uint32_t acc[G::R];
  constexpr bool REG_XOR = EncShape<ID>::reg_xor;
  const size_t nw = (size_t)G::U_WORDS;

  if constexpr (MODE == ENC_CODE) {
    // C.Encode (Sec. II-A) with an optional symbol-error pattern added
    // between the outer and the inner code: RS codeword of m, + sym_err,
    // then each RS symbol as a duplicated RM(1,7) block; stored straight
    // from registers (lane-strided, coalesced)
    const uint8_t *mrow = a.m + (size_t)item * G::k;
    const uint32_t mlane = lane < G::k ? (uint32_t)mrow[lane] : 0u;
    rs_codeword<ID>(mlane, sym);
    wave_sync();
    if (a.sym_err) {
      const uint8_t *er = a.sym_err + (size_t)item * G::n1;
      for (int j = lane; j < G::n1; j += 64) sym[j] ^= er[j];
      wave_sync();
    }
    uint32_t *dst = (uint32_t *)(a.v_out + (size_t)item * G::V_WORDS);
#pragma unroll 4
    for (int i = 0; i < (G::W32 + 63) / 64; ++i) {
      const int d = lane + 64 * i;
      const int dd = d < G::W32 ? d : 0;
      const int blk = dd / G::BLK, w = (dd % G::BLK) & 3;
      const uint32_t word = rm_dword(sym[blk], (uint32_t)w, pat);
      if (d < G::W32) dst[d] = word;
    }
    wave_sync();  // the symbol table is rewritten by the next item
    return;
  } else if constexpr (MODE == ENC_SAMPLE) {
    constexpr int WR = Set<ID>::wr, WE = Set<ID>::we;
    static_assert(WR == WE, "one sampling loop for r1, r2 and e");
    uint32_t sp[3][(WR + 63) / 64];
    load_draws<WR>(a.draws + (size_t)item * a.draw_stride, sp);
    floyd3<ID, WR>(sp);
    const auto &ir1 = sp[0], &ir2 = sp[1], &ie = sp[2];
    uint32_t *out = a.supp_out + (size_t)item * (2 * WR + WE);
#pragma unroll
    for (int c = 0; c < (WR + 63) / 64; ++c) {
      const int i = 64 * c + lane;
      if (i < WR) {
        out[i] = ir1[c];
        out[WR + i] = ir2[c];
      }
    }
#pragma unroll
    for (int c = 0; c < (WE + 63) / 64; ++c) {
      const int i = 64 * c + lane;
      if (i < WE) out[2 * WR + i] = ie[c];
    }
    return;
  } else if constexpr (MODE == ENC_KEYGEN) {
    // Alg. 3: s = x + h*y
    constexpr int NR = (G::w + 63) / 64;
    uint32_t iy[NR], ix[NR];
    load_support<G::w>(a.y + (size_t)item * G::w, iy);
    load_support<G::w>(a.x + (size_t)item * G::w, ix);
    // hr holds this item's h (loaded during the previous item when
    // pipelined) and receives the next item's h while h*y is computed
    constexpr bool KPIPE = EncShape<ID>::keygen_pipe;
    if constexpr (!KPIPE) load_dense<ID>(a.h + item * nw, hr);
    build_doubled_regs<ID, kDenseRegs<ID>>(u2, hr);
    wave_sync();
    if (KPIPE && next < a.count) load_dense<ID>(a.h + (size_t)next * nw, hr);
    sparse_product<ID, G::w, EncShape<ID>::keygen_pipelined>(u2, iy, acc);
    if constexpr (REG_XOR) sparse_xor<ID, G::w>(acc, ix, (uint32_t)G::n);
    wave_sync();  // every window of U2 has been read
    put_full<ID>(buf, acc);
    if constexpr (!REG_XOR) lds_sparse_xor<ID, G::w>(buf, ix, (uint32_t)G::n);
    wave_sync();
    emit(buf, G::DW + 1, 2 * G::U_WORDS, a.s_out + item * nw);
    wave_sync();
    return;
  } else {
    // encryption.  Pipelined: hr holds this item's h, loaded during the
    // previous item, and receives the next item's h while s*r2 is computed;
    // s is loaded while h is staged and the supports are sampled.  Else
    // each row is loaded where it is used.
    constexpr bool PIPE = EncShape<ID>::pipe;
    constexpr int WR = Set<ID>::wr, WE = Set<ID>::we;
    constexpr bool CHECK = MODE == ENC_CHECK;
    static_assert(WR == WE, "one sampling loop for r1, r2 and e");
    uint32_t sp[3][(WR + 63) / 64];
    auto &ir1 = sp[0], &ir2 = sp[1], &ie = sp[2];
    if constexpr (MODE == ENC_ARRAYS) {
      load_support<WR>(a.r1 + (size_t)item * WR, ir1);
      load_support<WR>(a.r2 + (size_t)item * WR, ir2);
      load_support<WE>(a.e + (size_t)item * WE, ie);
    } else {
      load_draws<WR>(a.draws + (size_t)item * a.draw_stride, sp);
    }
    const uint8_t *mrow = a.m + (size_t)item * G::k;
    const uint32_t mlane = lane < G::k ? (uint32_t)mrow[lane] : 0u;  // byte t of m in lane t
    uint32_t sr[kDenseRegs<ID>];
    if constexpr (PIPE) {
      load_dense<ID>(a.s + item * nw, sr);
    } else {
      load_dense<ID>(a.h + item * nw, hr);
    }
    // the check's received u, loaded while h*r2 is computed
    constexpr bool AHEAD = CHECK && EncShape<ID>::check_ahead;
    constexpr int UOUT = 2 * G::U_WORDS;
    uint32_t cu[CHECK ? (UOUT + 63) / 64 : 1];
    if constexpr (AHEAD) load_row<UOUT>(a.u_in + item * nw, cu);
    build_doubled_regs<ID, kDenseRegs<ID>>(u2, hr);
    wave_sync();
    if constexpr (MODE != ENC_ARRAYS) floyd3<ID, WR>(sp);
    // Alg. 1: u = r1 + h*r2
    sparse_product<ID, WR>(u2, ir2, acc);
    if constexpr (REG_XOR) sparse_xor<ID, WR>(acc, ir1, (uint32_t)G::n);
    wave_sync();  // every window of U2 has been read
    put_full<ID>(buf, acc);
    if constexpr (!REG_XOR) lds_sparse_xor<ID, WR>(buf, ir1, (uint32_t)G::n);
    wave_sync();
    uint32_t diff = 0;
    if constexpr (CHECK) {
      if constexpr (!AHEAD) load_row<UOUT>(a.u_in + item * nw, cu);
      diff = compare_row<UOUT>(buf, G::DW + 1, cu);
    } else
      emit(buf, G::DW + 1, UOUT, a.u_out + item * nw);
    wave_sync();
    // the check's received v, loaded while s*r2 is computed (before the next
    // item's h, so that waiting for it does not wait for those)
    uint32_t cv[CHECK ? (G::W32 + 63) / 64 : 1];
    if constexpr (AHEAD) load_row<G::W32>(a.v_in + item * (size_t)G::V_WORDS, cv);

    // the RS codeword of m: parity, then the message
    rs_codeword<ID>(mlane, sym);

    // v = mG + s*r2 + e, first n1*n2 bits
    wave_sync();
    if constexpr (!PIPE) load_dense<ID>(a.s + item * nw, sr);
    build_doubled_regs<ID, kDenseRegs<ID>>(u2, sr);
    wave_sync();
    if (PIPE && next < a.count) load_dense<ID>(a.h + (size_t)next * nw, hr);
    sparse_product<ID, WR>(u2, ir2, acc);
    if constexpr (REG_XOR) sparse_xor<ID, WE>(acc, ie, (uint32_t)(G::n1 * G::n2));
    wave_sync();  // every window of U2 has been read
    // an opaque copy of the lane number: the per-register offsets below are
    // recomputed here rather than hoisted out of the item loop and kept live
    int ln = lane;
    asm volatile("" : "+v"(ln));
#pragma unroll
    for (int j = 0; j < G::R; ++j) {
      const int d = Layout<G>::out(ln, j);
      const int dd = d < G::W32 ? d : 0;
      const int blk = dd / G::BLK, w = (dd % G::BLK) & 3;
      const uint32_t word = rm_dword(sym[blk], (uint32_t)w, pat);
      if (d < G::W32) buf[d] = acc[j] ^ word;
    }
    if constexpr (!REG_XOR) lds_sparse_xor<ID, WE>(buf, ie, (uint32_t)(G::n1 * G::n2));
    wave_sync();
    if constexpr (CHECK) {
      if constexpr (!AHEAD) load_row<G::W32>(a.v_in + item * (size_t)G::V_WORDS, cv);
      diff |= compare_row<G::W32>(buf, G::W32, cv);
    } else
      emit(buf, G::W32, G::W32, a.v_out + item * (size_t)G::V_WORDS);
    if constexpr (CHECK) {
      const bool same = __ballot(diff != 0u) == 0ull;
      if (lane == 0) a.ok[item] = same ? 1u : 0u;
    }
    wave_sync();
  }
}

template <int MODE, int ID>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MODE == ENC_STREAM || MODE == ENC_CHECK ? EncShape<ID>::sampled_waves
                                   : MODE == ENC_KEYGEN                     ? EncShape<ID>::keygen_waves
                                                                            : EncShape<ID>::waves))) void
hqc_encrypt_kernel(EncArgs a) {
  extern __shared__ uint32_t lds[];
  using G = Geo<ID>;
  const int lane = lane_id();
  const uint32_t pat = rm_pattern((uint32_t)lane & 31u);
  uint32_t hr[kDenseRegs<ID>];
  constexpr bool AHEAD = MODE == ENC_KEYGEN ? EncShape<ID>::keygen_pipe
                                            : MODE != ENC_SAMPLE && MODE != ENC_CODE &&
                                                  EncShape<ID>::pipe;
  if (AHEAD && blockIdx.x < a.count) load_dense<ID>(a.h + (size_t)blockIdx.x * G::U_WORDS, hr);
  for (uint32_t item = blockIdx.x; item < a.count; item += gridDim.x)
    run_item<ID, MODE>(a, item, item + gridDim.x, lds, pat, hr);
}

template <int ID> size_t enc_lds() { return Layout<Geo<ID>>::ENC_LDS_BYTES; }

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
    case ENC_SAMPLE: return enc_ptr<ENC_SAMPLE>(pid);
    case ENC_CODE: return enc_ptr<ENC_CODE>(pid);
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
