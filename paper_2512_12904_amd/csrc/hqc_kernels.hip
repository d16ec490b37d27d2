// hqc_kernels.hip -- fused HQC.PKE.Decrypt for gfx950 (CDNA4).
//
// One workgroup = one 64-lane wavefront.  The grid is persistent: workgroup
// g takes tiles g, g + G, g + 2G, ... of the launch; a tile is up to 64
// consecutive items of one parameter set (a public property of the item, so
// the branch on it is uniform and independent of secret data).
//
// Per item of a tile, all 64 lanes cooperate:
//  S0  u is staged in LDS as a bit-level doubled copy U2[t] = u[t mod n],
//      t < 2n, so that every rotation of u is a contiguous window of U2.
//  S1  u*y (Eq. (1)): for support index y_k, output dword d of the product is
//      the 32 bits of U2 starting at bit 32d + n - y_k: one funnel shift
//      (v_alignbit_b32) of two adjacent U2 dwords.  Lane l owns the R
//      consecutive output dwords from l*R (R odd, so the 64 lanes' windows
//      fall in distinct LDS banks whatever the secret offset is).  The next
//      index's window is loaded while the current one is combined.
//  S2  XOR with v, into an LDS copy of v laid out one RM block per padded row.
//  S3-S5  one RM block per lane pair, 32 per pass: bit-sliced sum of the
//      copies, the 128-point Walsh-Hadamard transform of the counts as an
//      int8 matrix product on the matrix cores (MFMA), and a packed 16-bit
//      peak search (magnitude, then smallest index, then sign); the symbol
//      byte goes to the tile's symbol table in LDS.
// Then each lane, or each lane pair for tiles of at most 32 items, decodes
// the Reed-Solomon word of one item of the tile (S6-S10): syndromes as
// GF(2)-linear bit rows, Berlekamp-Massey in its reformulated form on
// bit-sliced vectors (2*delta steps), the error evaluator by a Horner
// scheme on the same planes, and Chien search + Forney at the k message
// positions only (the parity positions never reach m).  The few products of
// two variables go through the log and exp tables, held in lanes 0..31 (8
// bytes per lane) and read with ds_bpermute_b32 from source lanes below 32,
// so no two lanes reading different entries share an LDS bank; a zero
// operand is carried as a log value >= 512 and masked.
//
// Constant time: loop bounds and branches depend only on the parameter set,
// the tile size and loop counters; secret values flow only through selects,
// bit masks, funnel-shift amounts, uniform LDS window offsets and bpermute
// indices into 32 source lanes.
#include "hqc_device.h"

namespace hqc {
namespace {

// ---- S3-S5: one duplicated RM(1,7) block -> symbol byte, on the matrix cores --
// Maximum-likelihood decoding of a block: the correlations of the received
// copies with the 256 codewords of RM(1,7) are +-(128 MULT [u == 0] - 2 H(u)),
// where H = W F is the Walsh-Hadamard transform of the copy counts F (the
// number of copies with bit k set; W[u][k] = (-1)^popcount(u & k)).  For the
// 32 blocks of a pass that is a dense 128 x 128 by 128 x 32 integer product,
// run as int8 MFMAs (v_mfma_i32_32x32x32_i8: 32 rows u of W times 32
// positions k, times the counts of 32 blocks, one block per column) -- 16
// per pass, in place of 7 stages of packed 16-bit butterflies (measured
// 10 % faster on the HQC-1 decryption, 15 % on the decoder stress launch).
// Lanes l and l + 32 hold block l mod 32 and both return its symbol.
//
// Positions are split over the four K steps t and the two half-waves h as
// k = 32 t + 16 h + c: byte c (0 .. 15) of lane (j, h)'s B operand in step t
// is F(32 t + 16 h + c) of block j -- the 16 bits 16h .. 16h + 15 of dword t
// of the bit-sliced counts, spread to bytes.  The A operand of lane (i, h) in
// M tile mt (rows u = 32 mt + i) and step t is then
// W[32 mt + i][32 t + 16 h + c] = (-1)^(popcount(i & (16 h + c)) + popcount(mt & t)):
// one per-lane tile A0 and its negation, chosen per (mt, t) at compile time.
// The result of M tile mt in lane (j, h), register 4 rb + ri, is H(u) of
// block j for u = 32 mt + 8 rb + 4 h + ri.
//
// The ML symbol is the smallest u maximising |H'(u)|, H'(u) = H(u) -
// 64 MULT [u == 0], with bit 7 = [H'(u) > 0].  The search runs on 16-bit
// pairs of results with two maxima, one per codeword sign, of the keys
// q * 128 + (127 - u) (q = +-H'(u), halved for MULT 5): one v_pk_mad_i16
// and one v_pk_max_i16 per sign and pair (HQC-1 65,536 decryptions -1.5 %,
// decoder stress -3 % against a single key of |H'|, sign and index).
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

// a * b + c on both 16-bit halves in one instruction (c from a scalar
// register: the per-pair constants stay out of VGPRs)
__device__ __forceinline__ s16x2 pk_mad_i16(s16x2 a, s16x2 b, uint32_t c) {
  uint32_t d;
  asm("v_pk_mad_i16 %0, %1, %2, %3"
      : "=v"(d)
      : "v"(__builtin_bit_cast(uint32_t, a)), "v"(__builtin_bit_cast(uint32_t, b)), "s"(c));
  return __builtin_bit_cast(s16x2, d);
}

template <int MULT>
__device__ __forceinline__ uint32_t rm_decode_mfma(const uint32_t *blk) {
  // an opaque copy of the lane number: A0 and the lane's shifts are rebuilt
  // here (a dozen instructions) rather than hoisted and kept live
  int lane = lane_id();
  asm volatile("" : "+v"(lane));
  const uint32_t h = (uint32_t)lane >> 5, i = (uint32_t)lane & 31u;
  // bit-sliced counts of the four dwords (positions 32t .. 32t + 31); the
  // lane keeps its 16 bits, moved down to bits 0 .. 15
  uint32_t p0[4], p1[4], p2[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const uint32_t x = blk[t], y = blk[4 + t], z = blk[8 + t];
    const uint32_t sm = xor3(x, y, z), cy = maj3(x, y, z);
    if constexpr (MULT == 3) {
      p0[t] = sm;
      p1[t] = cy;
      p2[t] = 0;
    } else {
      const uint32_t d = blk[12 + t], f = blk[16 + t];
      const uint32_t sm2 = xor3(sm, d, f), cy2 = maj3(sm, d, f);
      p0[t] = sm2;
      p1[t] = cy ^ cy2;
      p2[t] = cy & cy2;
    }
    p0[t] >>= 16 * h;
    p1[t] >>= 16 * h;
    p2[t] >>= 16 * h;
  }
  // B operands: byte c of step t = F(32 t + 16 h + c); a nibble of a plane
  // spreads to the low bit of 4 bytes by one multiply
  i32x4 B[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      uint32_t v = (__builtin_amdgcn_ubfe(p0[t], 4 * d, 4) * 0x204081u) & 0x01010101u;
      v += ((__builtin_amdgcn_ubfe(p1[t], 4 * d, 4) * 0x204081u) & 0x01010101u) << 1;
      if constexpr (MULT == 5)
        v += ((__builtin_amdgcn_ubfe(p2[t], 4 * d, 4) * 0x204081u) & 0x01010101u) << 2;
      B[t][d] = (int)v;
    }
  // A0: byte c = (-1)^(popcount(i & c) + i_4 h) as int8.  For c = 4 d + e,
  // popcount(i & c) = popcount(i & 4d) + popcount(i & e): dword d is the
  // pattern of e = 0 .. 3 with every byte negated where parity(i & 4d)
  // (negation of +-1 bytes: XOR 0xFE)
  const uint32_t par_e = ((i & 1u) ? 0x0000FF00u | 0xFF000000u : 0u) ^
                         ((i & 2u) ? 0x00FF0000u | 0xFF000000u : 0u);
  const uint32_t flip = ((i >> 4) & h) ? 0xFEFEFEFEu : 0u;
  const uint32_t w0 = (0x01010101u ^ (par_e & 0xFEFEFEFEu)) ^ flip;
  const uint32_t m2 = (i & 4u) ? 0xFEFEFEFEu : 0u, m3 = (i & 8u) ? 0xFEFEFEFEu : 0u;
  const i32x4 A0 = {(int)w0, (int)(w0 ^ m2), (int)(w0 ^ m3), (int)(w0 ^ m2 ^ m3)};
  const i32x4 An = A0 ^ (int)0xFEFEFEFEu;
  // two running maxima of 16-bit keys q * 128 + (127 - u): q = H'(u) for
  // the codewords of sign + (pmax) and q = -H'(u) for sign - (nmax); for
  // MULT 5 q is halved first (H' up to 320; every H'(u) of a block has the
  // parity of sum F, so halving keeps the order, and -H' >> 1 is
  // par - (H' >> 1) with par = -1 for odd H', 0 for even)
  const s16x2 kmin = {-32768, -32768};
  s16x2 pmax = kmin, nmax = kmin;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    i32x16 acc = {};
#pragma unroll
    for (int t = 0; t < 4; ++t)
      acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_popcount(mt & t) & 1 ? An : A0, B[t],
                                                  acc, 0, 0, 0);
    // H'(0) = H(0) - 64 MULT (u = 0: tile 0, register 0 of the lower half)
    if (mt == 0) acc[0] -= h ? 0 : 64 * MULT;
    const short par = (acc[0] & 1) ? (short)-1 : (short)0;
    const s16x2 parv = {par, par};
    // registers v and v + 4 (u and u + 8) as one 16-bit pair; the keys carry
    // 127 - u with the half's 4 h left out (dropped from the maxima below)
#pragma unroll
    for (int rb = 0; rb < 4; rb += 2)
#pragma unroll
      for (int ri = 0; ri < 4; ++ri) {
        const int v = 4 * rb + ri;
        const uint32_t ulo = (uint32_t)(32 * mt + 8 * rb + ri);
        const uint32_t idx = (127u - ulo) | (119u - ulo) << 16;
        const s16x2 hv =
            __builtin_bit_cast(s16x2, __builtin_amdgcn_perm((uint32_t)acc[v + 4], (uint32_t)acc[v], 0x05040100u));
        const s16x2 c128 = {128, 128}, cm128 = {-128, -128};
        s16x2 kp, kn;
        if constexpr (MULT == 3) {
          kp = pk_mad_i16(hv, c128, idx);
          kn = pk_mad_i16(hv, cm128, idx);
        } else {
          const s16x2 q = hv >> (short)1;
          kp = pk_mad_i16(q, c128, idx);
          kn = pk_mad_i16(parv - q, c128, idx);
        }
        pmax = __builtin_elementwise_max(pmax, kp);
        nmax = __builtin_elementwise_max(nmax, kn);
      }
  }
  // the lane's best of each sign, then the sign of the larger (the winner's
  // |H'| is never 0, so the two never tie); bit 0 of the key = [H' > 0]
  const int p = (pmax.x > pmax.y ? pmax.x : pmax.y) - 4 * (int)h;
  const int q = (nmax.x > nmax.y ? nmax.x : nmax.y) - 4 * (int)h;
  const int mine = p >= q ? 2 * p + 1 : 2 * q;
  const Halves both = halves((uint32_t)mine);
  const int lo = (int)both.lo, hi = (int)both.hi;
  const uint32_t best = (uint32_t)(lo > hi ? lo : hi);
  return (127u - ((best >> 1) & 127u)) | (best & 1u) << 7;
}

// ---- S0-S2: received word r = v + (u*y)|_{n1 n2} into the padded rows -------

// One item's inputs, loaded lane-strided into VGPRs ahead of use so that the
// HBM latency of item i+1 overlaps the RM decoding of item i.
template <int ID> struct ItemRegs {
  using G = Geo<ID>;
  static constexpr int UREG = (G::DW + 1 + 63) / 64;  // u dwords 0 .. DW
  static constexpr int VREG = (G::W32 + 63) / 64;
  uint32_t u[UREG];
  uint32_t v[VREG];
  uint32_t y[G::YREG];
};

template <int ID, int OP, int SH>
__device__ __forceinline__ void prefetch(const SegDev &sg, uint32_t item, ItemRegs<ID> &r) {
  using G = Geo<ID, SH>;
  using IR = ItemRegs<ID>;
  const int lane = lane_id();
  const uint32_t *vsrc = (const uint32_t *)((OP == OP_DECODE ? sg.u : sg.v) +
                                            (size_t)item * G::V_WORDS);
  {  // v with u and y (the compact layout keeps it until the product is done)
#pragma unroll
    for (int i = 0; i < IR::VREG; ++i) {
      const int d = lane + 64 * i;
      r.v[i] = d < G::W32 ? vsrc[d] : 0u;
    }
  }
  if constexpr (OP != OP_DECODE) {
    const uint32_t *usrc = (const uint32_t *)(sg.u + (size_t)item * G::U_WORDS);
#pragma unroll
    for (int i = 0; i < IR::UREG; ++i) {
      const int d = lane + 64 * i;
      r.u[i] = d <= G::DW ? usrc[d] : 0u;
    }
    uint32_t key = 0;
    if constexpr (OP == OP_KEYED) {
      key = __builtin_amdgcn_readfirstlane(sg.key_ids[item]);
      key = key < sg.ks_cap ? key : 0u;  // out-of-range ids decrypt to zeros later
    }
    const uint32_t *ysrc =
        (OP == OP_KEYED) ? sg.ks_y + (size_t)key * G::w : sg.y + (size_t)item * G::w;
#pragma unroll
    for (int c = 0; c < G::YREG; ++c) {
      const int idx = 64 * c + lane;
      r.y[c] = idx < G::w ? ysrc[idx] : 0u;
    }
  }
}

// The received word of one item from its registers r; once r is consumed
// (before the product), the next item's loads are issued into r when
// `next` is set, so that they overlap this item's product and RM passes.
template <int ID, int OP, int SH>
__device__ __forceinline__ void received_word(ItemRegs<ID> &r, uint32_t *lds, uint32_t *rb,
                                              const uint32_t *vsrc, const SegDev &sg,
                                              uint32_t next_item, bool next) {
  using G = Geo<ID, SH>;
  using L = Layout<G>;
  using IR = ItemRegs<ID>;
  const int lane = lane_id();
  uint32_t *u2 = lds;

  if (!G::COMPACT || OP == OP_DECODE) {
#pragma unroll
    for (int i = 0; i < IR::VREG; ++i) {
      const int d = lane + 64 * i;
      if (d < G::W32) rb[L::row(d)] = r.v[i];
    }
  }
  if constexpr (OP == OP_DECODE) {
    if (next) prefetch<ID, OP, SH>(sg, next_item, r);
    return;
  }

  // S0: U2[0 .. DW) = u, then U2[DW ..] = the wrapped continuation
  // U2[t] = u[t - n], from the registers
  build_doubled_regs<ID, IR::UREG>(u2, r.u);
  uint32_t shreg[G::YREG];
  window_shifts<ID, G::YREG>(r.y, shreg);
  if (next) prefetch<ID, OP, SH>(sg, next_item, r);
  wave_sync();

  // S1: product, R output dwords per lane
  uint32_t acc[G::R];
#pragma unroll
  for (int j = 0; j < G::R; ++j) acc[j] = 0;
  product_acc<ID, G::w>(u2, shreg, acc);
  // S2: r = v + (u*y) restricted to the first n1*n2 bits
  if constexpr (G::COMPACT) {
    wave_sync();  // every window of U2 has been read: the rows take its place
#pragma unroll
    for (int j = 0; j < G::R; ++j) {
      const int d = L::out(lane, j);
      if (d < G::W32) rb[L::row(d)] = acc[j];
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < IR::VREG; ++i) {
      const int d = lane + 64 * i;
      if (d < G::W32) rb[L::row(d)] ^= r.v[i];
    }
  } else {
#pragma unroll
    for (int j = 0; j < G::R; ++j) {
      const int d = L::out(lane, j);
      if (d < G::W32) rb[L::row(d)] ^= acc[j];
    }
  }
}

// ---- GF(2)-linear steps of S6 and S8-S10 as bit rows -------------------------
// A sum of the word's bytes times fixed field elements is GF(2)-linear in the
// bits of those bytes: it is the XOR of one fixed row per set bit, row (j, b)
// being alpha^b times the constants that byte j is multiplied by.  The rows
// are the same for every lane, so they are read into scalar registers; each
// bit becomes an all-ones or all-zero mask that selects its row.  The
// syndromes and the Chien / Forney evaluations thus read no table at a
// word-dependent index and cost two VALU operations per bit and dword of
// results.
template <int NR, int Q> struct BitRows {
  uint32_t r[NR][8][Q];
};

struct GfPow {
  uint8_t e[255];
};
constexpr GfPow make_gf_pow() {
  GfPow t{};
  unsigned x = 1;
  for (int i = 0; i < 255; ++i) {
    t.e[i] = (uint8_t)x;
    x <<= 1;
    if (x & 0x100u) x ^= 0x11Du;
  }
  return t;
}

// syndrome rows: byte t of dword q of row (j, b) is alpha^(b + i j) for the
// syndrome index i = 4q + t + 1 <= NS.  The one-lane form computes all
// 2 delta syndromes (NS = 2 delta), the lane-pair form the first delta in
// each half (NS = delta); each form has its own table so that a row is one
// contiguous block of scalar loads.
template <int ID, int NS> struct SynShape {
  static constexpr int Q = (NS + 3) / 4;
  using T = BitRows<Geo<ID>::n1, Q>;
};
template <int ID> using SynLane = SynShape<ID, Geo<ID>::TD>;
template <int ID> using SynPair = SynShape<ID, Geo<ID>::TD / 2>;
template <int ID, int NS> constexpr typename SynShape<ID, NS>::T make_syn_rows() {
  using Sh = SynShape<ID, NS>;
  typename Sh::T t{};
  const GfPow g = make_gf_pow();
  for (int j = 0; j < Geo<ID>::n1; ++j)
    for (int b = 0; b < 8; ++b)
      for (int q = 0; q < Sh::Q; ++q) {
        uint32_t w = 0;
        for (int u = 0; u < 4; ++u) {
          const int i = 4 * q + u + 1;
          if (i <= NS) w |= (uint32_t)g.e[(b + i * j) % 255] << (8 * u);
        }
        t.r[j][b][q] = w;
      }
  return t;
}

// evaluation rows at the message positions X = alpha^(TD + t), t < k: byte u
// of dword p of row (e, b) is alpha^(b - e (TD + 4p + u)), the factor of bit
// b of coefficient e of Lambda or Omega in its value at X^-1
template <int ID> struct EvalShape {
  static constexpr int P = Geo<ID>::k / 4;
  using T = BitRows<Geo<ID>::TD + 1, P>;
};
template <int ID> constexpr typename EvalShape<ID>::T make_eval_rows() {
  using G = Geo<ID>;
  typename EvalShape<ID>::T t{};
  const GfPow g = make_gf_pow();
  for (int e = 0; e <= G::TD; ++e)
    for (int b = 0; b < 8; ++b)
      for (int p = 0; p < EvalShape<ID>::P; ++p) {
        uint32_t w = 0;
        for (int u = 0; u < 4; ++u) {
          const int j = G::TD + 4 * p + u;
          w |= (uint32_t)g.e[((b - e * j) % 255 + 255) % 255] << (8 * u);
        }
        t.r[e][b][p] = w;
      }
  return t;
}

// multiplication by alpha^(delta j) as bit rows: byte b % 4 of dword b / 4 of
// row j is alpha^(delta j + b), the image of bit b of a symbol
template <int ID> struct PremulRows {
  uint32_t r[Geo<ID>::n1][2];
};
template <int ID> constexpr PremulRows<ID> make_premul_rows() {
  PremulRows<ID> t{};
  const GfPow g = make_gf_pow();
  for (int j = 0; j < Geo<ID>::n1; ++j)
    for (int b = 0; b < 8; ++b)
      t.r[j][b / 4] |= (uint32_t)g.e[((Geo<ID>::TD / 2) * j + b) % 255] << (8 * (b % 4));
  return t;
}
__constant__ PremulRows<1> kPremul1 = make_premul_rows<1>();
__constant__ PremulRows<3> kPremul3 = make_premul_rows<3>();
__constant__ PremulRows<5> kPremul5 = make_premul_rows<5>();
template <int ID> __device__ __forceinline__ const PremulRows<ID> &premul_rows() {
  if constexpr (ID == 1) return kPremul1;
  else if constexpr (ID == 3) return kPremul3;
  else return kPremul5;
}

// (HQC-5 always decodes on lane pairs: no one-lane table)
__constant__ SynLane<1>::T kSynL1 = make_syn_rows<1, Geo<1>::TD>();
__constant__ SynLane<3>::T kSynL3 = make_syn_rows<3, Geo<3>::TD>();
__constant__ SynPair<1>::T kSynP1 = make_syn_rows<1, Geo<1>::TD / 2>();
__constant__ SynPair<3>::T kSynP3 = make_syn_rows<3, Geo<3>::TD / 2>();
__constant__ SynPair<5>::T kSynP5 = make_syn_rows<5, Geo<5>::TD / 2>();
__constant__ EvalShape<1>::T kEval1 = make_eval_rows<1>();
__constant__ EvalShape<3>::T kEval3 = make_eval_rows<3>();
__constant__ EvalShape<5>::T kEval5 = make_eval_rows<5>();

template <int ID> __device__ __forceinline__ const typename SynLane<ID>::T &syn_rows_lane() {
  static_assert(ID != 5, "HQC-5 decodes on lane pairs");
  if constexpr (ID == 1) return kSynL1;
  else return kSynL3;
}
template <int ID> __device__ __forceinline__ const typename SynPair<ID>::T &syn_rows_pair() {
  if constexpr (ID == 1) return kSynP1;
  else if constexpr (ID == 3) return kSynP3;
  else return kSynP5;
}
template <int ID> __device__ __forceinline__ const typename EvalShape<ID>::T &eval_rows() {
  if constexpr (ID == 1) return kEval1;
  else if constexpr (ID == 3) return kEval3;
  else return kEval5;
}

// acc[q] ^= rows[b][q] for every set bit b of the byte x, q < NQ
template <int NQ, int Q>
__device__ __forceinline__ void add_rows(uint32_t (&acc)[NQ], uint32_t x,
                                         const uint32_t (&rows)[8][Q]) {
  static_assert(NQ <= Q, "rows cover the accumulators");
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)x, b, 1);
    // v_bitop3 truth table 0x6C: S1 ^ (S0 & S2)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = __builtin_amdgcn_bitop3_b32(rows[b][q], acc[q], m, 0x6C);
  }
}

__device__ __forceinline__ uint32_t byte_of(const uint32_t *a, int t) {
  return __builtin_amdgcn_ubfe(a[t >> 2], 8 * (t & 3), 8);
}

// ---- Bit-sliced GF(2^8) vectors ------------------------------------------------
// A vector of field elements is held as 8 bit planes: bit i of plane j is
// bit j of element i, NC dwords per plane (element i in dword i / 32).
// Multiplying the whole vector by a scalar c is sum_k c_k (alpha^k T), and
// alpha x on planes is a renaming plus three XORs (alpha^8 = alpha^4 +
// alpha^3 + alpha^2 + 1): 64 v_bitop3 and 21 XORs per 32 elements, with the
// scalar's bits as all-ones / all-zero masks and no table read.

// D ^= c T, cm[k] = the mask of bit k of c
template <int NC>
__device__ __forceinline__ void mul_acc(uint32_t (&D)[8][NC], const uint32_t (&T)[8][NC],
                                        const uint32_t (&cm)[8]) {
  uint32_t cur[8][NC];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int q = 0; q < NC; ++q) cur[j][q] = T[j][q];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    // truth table 0x6C: S1 ^ (S0 & S2)
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int q = 0; q < NC; ++q) D[j][q] = __builtin_amdgcn_bitop3_b32(cur[j][q], D[j][q], cm[k], 0x6C);
    if (k < 7) {
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const uint32_t c7 = cur[7][q];
        cur[7][q] = cur[6][q];
        cur[6][q] = cur[5][q];
        cur[5][q] = cur[4][q];
        cur[4][q] = cur[3][q] ^ c7;
        cur[3][q] = cur[2][q] ^ c7;
        cur[2][q] = cur[1][q] ^ c7;
        cur[1][q] = cur[0][q];
        cur[0][q] = c7;
      }
    }
  }
}

// o = a << 1 across NC dwords
template <int NC>
__device__ __forceinline__ void shl1(const uint32_t (&a)[NC], uint32_t (&o)[NC]) {
  o[0] = a[0] << 1;
#pragma unroll
  for (int q = 1; q < NC; ++q) o[q] = __builtin_amdgcn_alignbit(a[q], a[q - 1], 31);
}

// clear the bits of elements >= n
template <int NC>
__device__ __forceinline__ void keep_elems(uint32_t (&P)[8][NC], int n) {
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const uint32_t m = n >= 32 * (q + 1) ? ~0u : (n > 32 * q ? (1u << (n - 32 * q)) - 1u : 0u);
#pragma unroll
    for (int j = 0; j < 8; ++j) P[j][q] &= m;
  }
}

// masks of the 8 bits of element i (dword col of the planes, col public)
template <int NC>
__device__ __forceinline__ void elem_masks(const uint32_t (&P)[8][NC], bool upper, uint32_t off,
                                           uint32_t (&m)[8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j)
    m[j] = (uint32_t)__builtin_amdgcn_sbfe((int)((NC > 1 && upper) ? P[j][NC - 1] : P[j][0]), off, 1);
}

// ---- S7: Berlekamp-Massey on bit-sliced vectors --------------------------------
// Massey's recursion (Lambda <- Lambda + (Delta / b) x^s B, B <- Lambda and
// b <- Delta when 2L <= r - 1) with the discrepancies read from a vector,
// as in the reformulation of Sarwate and Shanbhag: they are not inner
// products but the low part of a vector D that is updated like Lambda.
// Massey's division by b (here gamma) is kept, so nothing is scaled.  With D holding
// S_1 .. S_2delta in region A and Lambda in region C (coefficient q at
// element q), step r is
//     Delta = D_A[r],  c = Delta / gamma,
//     U = swap ? D : T,  D <- D + c T,  T <- x U,
//     gamma <- swap ? Delta : gamma,
// swap = (Delta != 0 and 2L <= r), on both regions alike (T starts as x D).
// Region C then holds Massey's Lambda itself (Lambda_0 = 1, exactly the
// oracle's coefficients, decoder failures included).
// Elements of region A below r and of region C above 2 delta are never
// read; they only move upwards, so they never reach the live elements.
template <int NC>
__device__ __forceinline__ void bm_step(uint32_t (&D)[8][NC], uint32_t (&T)[8][NC],
                                        const uint32_t (&cm)[8], bool sw) {
  uint32_t U[8][NC];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int q = 0; q < NC; ++q) U[j][q] = sw ? D[j][q] : T[j][q];
  mul_acc(D, T, cm);
#pragma unroll
  for (int j = 0; j < 8; ++j) shl1(U[j], T[j]);
}

// element i of a planar vector as a byte (column col and offset off)
template <int NC>
__device__ __forceinline__ uint32_t plane_byte(const uint32_t (&P)[8][NC], int col, uint32_t off) {
  uint32_t b = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) b |= __builtin_amdgcn_ubfe(P[j][col], off, 1) << j;
  return b;
}

// Delta = element r of region A (r uniform), as a byte
template <int NC>
__device__ __forceinline__ uint32_t elem_byte(const uint32_t (&P)[8][NC], int r) {
  uint32_t d = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t w = (NC > 1 && r >= 32) ? P[j][NC - 1] : P[j][0];
    d |= __builtin_amdgcn_ubfe(w, (uint32_t)r & 31u, 1) << j;
  }
  return d;
}

// ---- S6-S10: Reed-Solomon decode of one item per lane ------------------------
template <int ID, int OP>
__device__ __forceinline__ void rs_lane(const SegDev &sg, uint32_t item, bool active,
                                        const uint8_t *cs, GfTab exp4, GfTab log4,
                                        uint8_t *dbg) {
  using G = Geo<ID>;
  constexpr int TD = G::TD;
  constexpr int P = EvalShape<ID>::P;
  constexpr int NCA = (TD + 31) / 32, NCC = (TD + 1 + 31) / 32;

  // S6: S_i = sum_j c_j alpha^(i j), i = 1 .. TD; byte i - 1 of sa (four to
  // a dword) is S_i
  uint32_t sa[SynLane<ID>::Q];
#pragma unroll
  for (int q = 0; q < SynLane<ID>::Q; ++q) sa[q] = 0;
#pragma unroll 1
  for (int j = 0; j < G::n1; ++j) add_rows(sa, (uint32_t)cs[j], syn_rows_lane<ID>().r[j]);
  if constexpr (OP == OP_DEBUG) {
    if (dbg) {
      for (int j = 0; j < G::n1; ++j) dbg[G::DBG_SYM + j] = cs[j];
#pragma unroll
      for (int i = 0; i < TD; ++i) dbg[G::DBG_S + i] = (uint8_t)byte_of(sa, i);
    }
  }
  // S(x) = sum_i S_i x^(i-1) as planes
  uint32_t SP[8][NCA];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
#pragma unroll
    for (int q = 0; q < NCA; ++q) SP[j][q] = 0;
#pragma unroll
    for (int m = 0; m < TD; ++m)
      SP[j][m >> 5] |= __builtin_amdgcn_ubfe(sa[m >> 2], 8 * (m & 3) + j, 1) << (m & 31);
  }

  // S7: region A = S_1 .. S_TD, region C = Lambda
  uint32_t DA[8][NCA], TA[8][NCA], DC[8][NCC], TC[8][NCC];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
#pragma unroll
    for (int q = 0; q < NCA; ++q) DA[j][q] = SP[j][q];
    shl1(SP[j], TA[j]);
#pragma unroll
    for (int q = 0; q < NCC; ++q) {
      DC[j][q] = (j == 0 && q == 0) ? 1u : 0u;
      TC[j][q] = (j == 0 && q == 0) ? 2u : 0u;
    }
  }
  {
    uint32_t lg = 0;  // log gamma
    int kk = 0;       // r - 2L
#pragma unroll 1
    for (int r = 0; r < TD; ++r) {
      const uint32_t d0 = elem_byte(DA, r);
      const uint32_t ld = logz(log4, d0);
      const uint32_t c = expz(exp4, ld + 255u - lg);
      const bool sw = d0 != 0 && kk >= 0;
      uint32_t cm[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) cm[k] = (uint32_t)__builtin_amdgcn_sbfe((int)c, k, 1);
      bm_step(DA, TA, cm, sw);
      bm_step(DC, TC, cm, sw);
      lg = sw ? (ld & 0xFFu) : lg;
      kk = sw ? -kk - 1 : kk + 1;
    }
  }
  keep_elems(DC, TD + 1);
  if constexpr (OP == OP_DEBUG) {
    if (dbg) {
#pragma unroll
      for (int i = 0; i <= TD; ++i)
        dbg[G::DBG_LAM + i] = (uint8_t)plane_byte(DC, i >> 5, (uint32_t)i & 31u);
    }
  }

  // S9 (part): Omega = S(x) Lambda(x) mod x^TD, by Horner over Lambda's
  // coefficients: W <- x W + Lambda_i S
  uint32_t W[8][NCA];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int q = 0; q < NCA; ++q) W[j][q] = 0;
#pragma unroll 1
  for (int i = TD; i >= 0; --i) {
    uint32_t lm[8];
    elem_masks(DC, i >= 32, (uint32_t)i & 31u, lm);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      uint32_t t[NCA];
      shl1(W[j], t);
#pragma unroll
      for (int q = 0; q < NCA; ++q) W[j][q] = t[q];
    }
    mul_acc(W, SP, lm);
  }
  keep_elems(W, TD);

  // S8 + S9: Lambda (even and odd parts) and Omega at X^-1 for the message
  // positions X = alpha^(TD + t): the bits of each coefficient select rows
  const auto &ev = eval_rows<ID>();
  uint32_t ae[P], ao[P], aw[P];
#pragma unroll
  for (int p = 0; p < P; ++p) ae[p] = ao[p] = aw[p] = 0;
#pragma unroll 1
  for (int i = 0; i <= TD; i += 2) {
    uint32_t lm[8], wm[8];
    elem_masks(DC, i >= 32, (uint32_t)i & 31u, lm);
    elem_masks(W, i >= 32, (uint32_t)i & 31u, wm);
    if (i == TD) {  // Omega has TD coefficients
#pragma unroll
      for (int b = 0; b < 8; ++b) wm[b] = 0;
    }
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int p = 0; p < P; ++p) {
        ae[p] = __builtin_amdgcn_bitop3_b32(ev.r[i][b][p], ae[p], lm[b], 0x6C);
        aw[p] = __builtin_amdgcn_bitop3_b32(ev.r[i][b][p], aw[p], wm[b], 0x6C);
      }
    if (i < TD) {
      const int i1 = i + 1;
      elem_masks(DC, i1 >= 32, (uint32_t)i1 & 31u, lm);
      elem_masks(W, i1 >= 32, (uint32_t)i1 & 31u, wm);
#pragma unroll
      for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int p = 0; p < P; ++p) {
          ao[p] = __builtin_amdgcn_bitop3_b32(ev.r[i1][b][p], ao[p], lm[b], 0x6C);
          aw[p] = __builtin_amdgcn_bitop3_b32(ev.r[i1][b][p], aw[p], wm[b], 0x6C);
        }
    }
  }

  // S10: Forney at message position j = TD + t, then m_t (four bytes of m
  // to a dword store)
  uint32_t pack = 0;
#pragma unroll
  for (int t = 0; t < G::k; ++t) {
    const uint32_t j = (uint32_t)(TD + t);
    const uint32_t oddv = byte_of(ao, t), omv = byte_of(aw, t);
    const uint32_t lamv = byte_of(ae, t) ^ oddv;
    // e_j = Omega(X^-1) / Lambda'(X^-1) with Lambda'(X^-1) = X * odd(X^-1), X = alpha^j
    const uint32_t x = red255(tab(log4, omv) + 255u - tab(log4, oddv));
    uint32_t e = tab(exp4, red255(x + 255u - j));
    e = (lamv == 0 && omv != 0 && oddv != 0) ? e : 0u;
    if constexpr (OP == OP_DEBUG)
      if (dbg) dbg[G::DBG_E + t] = (uint8_t)e;
    pack |= ((cs[j] ^ e) & 0xFFu) << (8 * (t & 3));
    if ((t & 3) == 3) {
      if (active) ((uint32_t *)(sg.m + (size_t)item * G::k))[t >> 2] = pack;
      pack = 0;
    }
  }
}

// ---- S6-S10 with two lanes per item (tiles of at most 32 items) ---------------
// Lanes l and l + 32 decode the same word.  Half h = l / 32 computes the
// syndromes S_{hH+1} .. S_{hH+H} (H = delta); in Berlekamp-Massey the lower
// half holds region A and the upper half region C, the discrepancy crossing
// through v_permlane32_swap_b32; half h then takes Lambda's and Omega's
// coefficients 2i + h for the evaluations.
template <int ID, int OP>
__device__ __forceinline__ void rs_pair(const SegDev &sg, uint32_t item, bool active,
                                        const uint8_t *cs, GfTab exp4, GfTab log4,
                                        uint8_t *dbg) {
  using G = Geo<ID>;
  constexpr int TD = G::TD;
  constexpr int H = TD / 2;
  constexpr int P = EvalShape<ID>::P;
  constexpr int NC = (TD + 1 + 31) / 32;
  static_assert(H < 32 && TD + 1 <= 64, "pair layout");
  const bool hi = lane_id() >= 32;
  const uint32_t h = hi ? 1u : 0u;

  // S6: this half's H syndromes.  The upper half first multiplies c_j by
  // alpha^(H j), so that S_{H+i} = sum_j (c_j alpha^(H j)) alpha^(i j) uses
  // the rows of S_i.
  constexpr int QP = (H + 3) / 4;
  uint32_t sa[QP];
#pragma unroll
  for (int q = 0; q < QP; ++q) sa[q] = 0;
  {
    const uint32_t base = hi ? (uint32_t)H : 0u;
#pragma unroll 1
    for (int j = 0; j < G::n1; ++j) {
      const uint32_t c = cs[j];
      // c alpha^(H j) by bit rows (a constant multiplier is GF(2)-linear)
      uint32_t m = 0;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint32_t row = __builtin_amdgcn_ubfe(premul_rows<ID>().r[j][b >> 2], 8 * (b & 3), 8);
        m = __builtin_amdgcn_bitop3_b32(row, m, (uint32_t)__builtin_amdgcn_sbfe((int)c, b, 1), 0x6C);
      }
      const uint32_t cp = hi ? m : c;
      add_rows(sa, cp, syn_rows_pair<ID>().r[j]);
    }
    if constexpr (OP == OP_DEBUG) {
      if (dbg) {
        if (!hi)
          for (int j = 0; j < G::n1; ++j) dbg[G::DBG_SYM + j] = cs[j];
#pragma unroll
        for (int i = 0; i < H; ++i) dbg[G::DBG_S + (int)base + i] = (uint8_t)byte_of(sa, i);
      }
    }
  }
  // S(x) = sum_i S_i x^(i-1) as planes, in both halves
  uint32_t SP[8][NC];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    uint32_t pl = 0;  // this half's syndromes, bit i <-> S_{hH+i+1}
#pragma unroll
    for (int i = 0; i < H; ++i) pl |= __builtin_amdgcn_ubfe(sa[i >> 2], 8 * (i & 3) + j, 1) << i;
    const Halves pv = halves(pl);
    SP[j][0] = pv.lo | (pv.hi << H);
    if constexpr (NC > 1) SP[j][1] = pv.hi >> (32 - H);
  }

  // S7: lower half region A = S_1 .. S_TD, upper half region C = Lambda
  uint32_t D[8][NC], T[8][NC];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    uint32_t ta[NC];
    shl1(SP[j], ta);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      D[j][q] = hi ? ((j == 0 && q == 0) ? 1u : 0u) : SP[j][q];
      T[j][q] = hi ? ((j == 0 && q == 0) ? 2u : 0u) : ta[q];
    }
  }
  {
    uint32_t lg = 0;  // log gamma
    int kk = 0;       // r - 2L
#pragma unroll 1
    for (int r = 0; r < TD; ++r) {
      const uint32_t d0 = halves(elem_byte(D, r)).lo;  // the lower half's element r
      const uint32_t ld = logz(log4, d0);
      const uint32_t c = expz(exp4, ld + 255u - lg);
      const bool sw = d0 != 0 && kk >= 0;
      uint32_t cm[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) cm[k] = (uint32_t)__builtin_amdgcn_sbfe((int)c, k, 1);
      bm_step(D, T, cm, sw);
      lg = sw ? (ld & 0xFFu) : lg;
      kk = sw ? -kk - 1 : kk + 1;
    }
  }
  // Lambda (the upper half's region C) in both halves
  uint32_t C[8][NC];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int q = 0; q < NC; ++q) C[j][q] = halves(D[j][q]).hi;
  keep_elems(C, TD + 1);
  if constexpr (OP == OP_DEBUG) {
    if (dbg && !hi) {
#pragma unroll
      for (int i = 0; i <= TD; ++i)
        dbg[G::DBG_LAM + i] = (uint8_t)plane_byte(C, i >> 5, (uint32_t)i & 31u);
    }
  }

  // S9 (part): Omega = S(x) Lambda(x) mod x^TD by Horner, W <- x W + Lambda_i S:
  // the lower half over i = H .. 0, the upper half over i = TD + 1 .. H + 1
  // (Lambda_{TD+1} = 0), whose sum is then multiplied by x^(H+1)
  uint32_t W[8][NC];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int q = 0; q < NC; ++q) W[j][q] = 0;
#pragma unroll 1
  for (int s = H; s >= 0; --s) {
    const uint32_t i = (uint32_t)s + (hi ? (uint32_t)(H + 1) : 0u);
    uint32_t lm[8];
    elem_masks(C, i >= 32u, i & 31u, lm);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      uint32_t t[NC];
      shl1(W[j], t);
#pragma unroll
      for (int q = 0; q < NC; ++q) W[j][q] = t[q];
    }
    mul_acc(W, SP, lm);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    uint32_t up[NC];  // W x^(H+1)
    up[0] = W[j][0] << (H + 1);
#pragma unroll
    for (int q = 1; q < NC; ++q) up[q] = __builtin_amdgcn_alignbit(W[j][q], W[j][q - 1], 31 - H);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const Halves wv = halves(hi ? up[q] : W[j][q]);
      W[j][q] = wv.lo ^ wv.hi;
    }
  }
  keep_elems(W, TD);

  // S8 + S9: P_h = sum_i Lambda_{2i+h} X^(-2i) and W_h = sum_i Omega_{2i+h}
  // X^(-2i) at the message positions, so that Lambda(X^-1) = P_0 + X^-1 P_1,
  // the odd part of Lambda at X^-1 is X^-1 P_1 and Omega(X^-1) = W_0 + X^-1 W_1
  const auto &ev = eval_rows<ID>();
  uint32_t al[P], aw[P];
#pragma unroll
  for (int p = 0; p < P; ++p) al[p] = aw[p] = 0;
#pragma unroll 1
  for (int i = 0; i <= H; ++i) {
    const bool upper = 2 * i >= 32;
    const uint32_t off = ((uint32_t)(2 * i) & 31u) + h;
    uint32_t lm[8], wm[8];
    elem_masks(C, upper, off, lm);
    elem_masks(W, upper, off, wm);
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int p = 0; p < P; ++p) {
        al[p] = __builtin_amdgcn_bitop3_b32(ev.r[2 * i][b][p], al[p], lm[b], 0x6C);
        aw[p] = __builtin_amdgcn_bitop3_b32(ev.r[2 * i][b][p], aw[p], wm[b], 0x6C);
      }
  }

  // S10: with X = alpha^j, Lambda'(X^-1) = X * odd(X^-1) = P_1, so the error
  // value is Omega(X^-1) / P_1 = (W_0 + X^-1 W_1) / P_1: half h contributes
  // W_h X^(-h) / P_1.  j is a root position when P_1 != 0 and
  // P_0 = X^-1 P_1.
  uint32_t pack = 0;
#pragma unroll
  for (int t = 0; t < G::k; ++t) {
    const uint32_t j = (uint32_t)(TD + t);
    const Halves lv = halves(logz(log4, byte_of(al, t)));  // log P_0, log P_1
    const uint32_t lw = red255(logz(log4, byte_of(aw, t)) + (hi ? 255u - j : 0u));
    const Halves tv = halves(expz(exp4, lw + 255u - (lv.hi & 0xFFu)));
    const bool root = lv.hi < ZL && lv.lo == red255(lv.hi + 255u - j);
    const uint32_t e = root ? (tv.lo ^ tv.hi) : 0u;
    if constexpr (OP == OP_DEBUG)
      if (dbg && !hi) dbg[G::DBG_E + t] = (uint8_t)e;
    pack |= ((cs[j] ^ e) & 0xFFu) << (8 * (t & 3));
    if ((t & 3) == 3) {
      if (active && !hi) ((uint32_t *)(sg.m + (size_t)item * G::k))[t >> 2] = pack;
      pack = 0;
    }
  }
}

// The RM symbols of nt <= TROWS consecutive items from item0 (S0-S5) into
// rows row0 .. row0 + nt - 1 of the symbol table.
template <int ID, int OP, int SH>
__device__ __forceinline__ void symbols(const SegDev &sg, uint32_t item0, int nt, int row0,
                                        uint32_t *lds) {
  using G = Geo<ID, SH>;
  using L = Layout<G>;
  const int lane = lane_id();
  uint8_t *const lds8 = (uint8_t *)lds;
  // the next item's u, v and y are loaded into VGPRs while this one's RM
  // blocks decode (HQC-1: already while its product runs); the compact
  // layout (HQC-5) loads each item's u, v and y together when it starts
  // (v too, so that its latency passes during the product: HQC-5 -11 %),
  // leaving the rest of the latency to the other wavefronts on the SIMD
  ItemRegs<ID> regs;
  if constexpr (!G::COMPACT) prefetch<ID, OP, SH>(sg, item0, regs);
  int passes = 0;  // RM passes done for the current group
  for (int it = 0; it < nt; ++it) {
    const uint32_t cur = item0 + (uint32_t)it;
    const int gi = it % G::RMG;  // slot of this item's received word
    if constexpr (G::COMPACT) prefetch<ID, OP, SH>(sg, cur, regs);
    // HQC-1 issues the next item's loads before this item's product (its
    // product is short: the loads would not be covered by RM passes alone);
    // HQC-3 after it (measured 1 % faster there)
    constexpr bool EARLY = ID == 1;
    received_word<ID, OP, SH>(regs, lds, lds + L::rb(gi),
                          (const uint32_t *)(sg.v + (size_t)cur * G::V_WORDS), sg, cur + 1,
                          EARLY && it + 1 < nt);
    wave_sync();
    if (OP == OP_DEBUG && sg.dbg) {  // debug launch: the received word, in item order
      const uint32_t *rb = lds + L::rb(gi);
      uint32_t *dst = (uint32_t *)(sg.dbg + (size_t)cur * G::DBG_BYTES);
      for (int d = lane; d < G::W32; d += 64) dst[d] = rb[L::row(d)];
    }
    if (!G::COMPACT && !EARLY && it + 1 < nt) prefetch<ID, OP, SH>(sg, cur + 1, regs);
    {
      // the group's blocks, flat index q n1 + b for block b of slot q, are
      // decoded BPP at a time (one lane or one lane pair each) as soon as the
      // received words holding them are complete, so that most items' loads
      // overlap a pass
      constexpr int BPP = L::BPP;
      const int g0 = it - gi, avail = (gi + 1) * G::n1;
      const bool last = gi == G::RMG - 1 || it == nt - 1;
      if (gi == 0) passes = 0;
#pragma unroll 1
      while (passes * BPP < avail && ((passes + 1) * BPP <= avail || last)) {
        const int fl = L::pass_flat(passes, lane);
        const int f = L::pass_clamp(fl, avail);
        const int q = f / G::n1, b = f - q * G::n1;
        const uint32_t *blk = lds + L::block(q, b);
        const uint32_t sbyte = rm_decode_mfma<G::MULT>(blk);
        if (fl < avail && lane < BPP) lds8[L::sym(row0 + g0 + q, b)] = (uint8_t)sbyte;
        ++passes;
      }
      wave_sync();
    }
  }
}

// Symbol-table rows whose Reed-Solomon words are still to be decoded: rows
// 0 .. fill - 1 of one segment, row r holding item row_item of lane r.
// Consecutive tiles of a workgroup fill it, and it is decoded in one pass
// (rs_flush) when the next tile would not fit in 32 rows, when the segment
// changes and at the end, so that a workgroup with several small tiles pays
// the Reed-Solomon stage's fixed cost per 32 words, not per tile.
struct Pending {
  int fill;
  uint32_t row_item;
};

// S6-S10 of the pending rows: one Reed-Solomon word per lane pair l, l + 32
// (at most 32 rows; always for the compact layout), or per lane (33 .. 64
// rows); lanes past the rows decode a copy of row 0 and store nothing
template <int ID, int OP, int SH>
__device__ __forceinline__ void rs_flush(const SegDev &sg, Pending &pd, uint32_t *lds, GfTab exp4,
                                         GfTab log4) {
  using G = Geo<ID, SH>;
  using L = Layout<G>;
  const int lane = lane_id();
  uint8_t *const lds8 = (uint8_t *)lds;
  const int nt = pd.fill;
  const bool pair = G::COMPACT || nt <= 32;
  const int s = pair ? (lane & 31) : lane;
  const int slot = s < nt ? s : 0;
  const uint32_t mine = pair ? halves(pd.row_item).lo : pd.row_item;  // item of row s
  const uint32_t item = s < nt ? mine : rdlane(pd.row_item, 0);
  bool active = s < nt;
  bool bad_key = false;
  if constexpr (OP == OP_KEYED) {
    bad_key = sg.key_ids[item] >= sg.ks_cap;
  }
  uint8_t *dbg = (OP == OP_DEBUG && sg.dbg && active) ? sg.dbg + (size_t)item * G::DBG_BYTES : nullptr;
  if constexpr (G::COMPACT) {
    rs_pair<ID, OP>(sg, item, active && !bad_key, lds8 + L::sym(slot, 0), exp4, log4, dbg);
  } else {
    if (pair)
      rs_pair<ID, OP>(sg, item, active && !bad_key, lds8 + L::sym(slot, 0), exp4, log4, dbg);
    else
      rs_lane<ID, OP>(sg, item, active && !bad_key, lds8 + L::sym(slot, 0), exp4, log4, dbg);
  }
  if constexpr (OP == OP_KEYED) {
    if (active && bad_key && s == lane) {
      for (int t = 0; t < G::k; ++t) sg.m[(size_t)item * G::k + t] = 0;
      atomicAdd(sg.ks_bad, 1ull);
    }
  }
  wave_sync();  // the rows are refilled after this
  pd.fill = 0;
}

// a tile of nt <= 64 items, in pieces of at most TROWS (32 for the compact
// layout): each piece's symbols go after the pending rows, which are decoded
// first when the piece would not fit in 32 rows; a piece of more than 32
// items is decoded at once (one word per lane)
template <int ID, int OP, int SH>
__device__ __forceinline__ void run_tile(const SegDev &sg, uint32_t item0, int nt, uint32_t *lds,
                                         GfTab exp4, GfTab log4, Pending &pd) {
  using G = Geo<ID, SH>;
  const int lane = lane_id();
  for (int s0 = 0; s0 < nt; s0 += G::TROWS) {
    const int sub = nt - s0 < G::TROWS ? nt - s0 : G::TROWS;
    if (pd.fill > 0 && pd.fill + sub > 32) rs_flush<ID, OP, SH>(sg, pd, lds, exp4, log4);
    const uint32_t first = item0 + (uint32_t)s0;
    symbols<ID, OP, SH>(sg, first, sub, pd.fill, lds);
    if (lane >= pd.fill && lane < pd.fill + sub) pd.row_item = first + (uint32_t)(lane - pd.fill);
    pd.fill += sub;
    if (pd.fill > 32) rs_flush<ID, OP, SH>(sg, pd, lds, exp4, log4);
  }
}

// shape 1 exists for single-set HQC-1 and HQC-3 kernels; SH 2 is the
// decoding kernels' shape 0 (no doubled u in LDS)
constexpr int kernel_waves(unsigned mask, int sh) {
  return sh == 2 ? Geo<5, 2>::WAVES
                 : sh == 1 ? (mask == 1u ? Geo<1, 1>::WAVES : Geo<3, 1>::WAVES) : 2;
}

// The tiles of segment s that this workgroup takes (units blockIdx.x,
// blockIdx.x + gridDim.x, ... that fall in the segment), Reed-Solomon rows
// pending across them and decoded at the end.
template <int ID, int OP, int SH>
__device__ __forceinline__ void run_segment(const KArgs &a, int s, uint32_t *lds, GfTab exp4,
                                            GfTab log4) {
  const SegDev &sg = a.seg[s];
  const uint32_t end = s + 1 < (int)a.nseg ? a.seg[s + 1].first : a.total;
  Pending pd{0, 0u};
  for (uint32_t unit = first_unit(blockIdx.x, gridDim.x, sg.first); unit < end;
       unit += gridDim.x) {
    const uint32_t item0 = (unit - sg.first) * sg.tile;
    const uint32_t left = sg.count - item0;
    const int nt = (int)(left < sg.tile ? left : sg.tile);
    run_tile<ID, OP, SH>(sg, item0, nt, lds, exp4, log4, pd);
  }
  if (pd.fill > 0) rs_flush<ID, OP, SH>(sg, pd, lds, exp4, log4);
}

template <int OP, unsigned MASK, int SH>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kernel_waves(MASK, SH)))) void
hqc_kernel(KArgs a) {
  static_assert(SH != 1 || MASK == 1u || MASK == 2u, "shape 1: HQC-1 or HQC-3 alone");
  static_assert(SH != 2 || OP == OP_DECODE, "the decoding layout keeps no doubled u");
  extern __shared__ uint32_t lds[];
  const GfTab exp4 = gf_exp_tab();
  const GfTab log4 = gf_log_tab();
  constexpr int SH1 = (MASK == 1u || SH == 2) ? SH : 0, SH3 = (MASK == 2u || SH == 2) ? SH : 0;
  constexpr int SH5 = SH == 2 ? 2 : 0;
  // the segment of each parameter set (each set appears at most once); the
  // sets run one after the other in straight-line code, so that no set's
  // loop-invariant registers stay live through another set's loop
  int s1 = -1, s3 = -1, s5 = -1;
  for (int s = 0; s < (int)a.nseg; ++s) {
    const int pid = a.seg[s].pid;
    s1 = pid == 1 ? s : s1;
    s3 = pid == 3 ? s : s3;
    s5 = pid == 5 ? s : s5;
  }
  if ((MASK & 1u) && s1 >= 0) run_segment<1, OP, SH1>(a, s1, lds, exp4, log4);
  if ((MASK & 2u) && s3 >= 0) run_segment<3, OP, SH3>(a, s3, lds, exp4, log4);
  if ((MASK & 4u) && s5 >= 0) run_segment<5, OP, SH5>(a, s5, lds, exp4, log4);
}

template <int OP>
const void *kernel_for_mask(unsigned mask, int shape) {
  if (shape == 1) {
    // debug launches run shape 0 only
    if constexpr (OP == OP_DEBUG) return nullptr;
    else if (mask == 1u) return (const void *)&hqc_kernel<OP, 1, 1>;
    else if (mask == 2u) return (const void *)&hqc_kernel<OP, 2, 1>;
    return nullptr;
  }
  // shape 0: decoding in its own layout (SH 2)
  constexpr int S0 = OP == OP_DECODE ? 2 : 0;
  switch (mask) {
    case 1: return (const void *)&hqc_kernel<OP, 1, S0>;
    case 2: return (const void *)&hqc_kernel<OP, 2, S0>;
    case 4: return (const void *)&hqc_kernel<OP, 4, S0>;
    default:
      // debug launches carry one parameter set: no mixed-set debug kernel
      if constexpr (OP == OP_DEBUG) return nullptr;
      else return (const void *)&hqc_kernel<OP, 7, S0>;
  }
}

template <int ID> void fill_info(SetInfo *o) {
  using G = Geo<ID>;
  o->n = G::n;
  o->n1 = G::n1;
  o->n2 = G::n2;
  o->k = G::k;
  o->delta = G::TD / 2;
  o->w = G::w;
  o->mult = G::MULT;
  o->u_words = G::U_WORDS;
  o->v_words = G::V_WORDS;
  o->lds_bytes = G::LDS_BYTES;
  o->dbg_bytes = G::DBG_BYTES;
  o->dbg_sym = G::DBG_SYM;
  o->dbg_s = G::DBG_S;
  o->dbg_lam = G::DBG_LAM;
  o->dbg_e = G::DBG_E;
}

}  // namespace

bool set_info(int pid, SetInfo *out) {
  switch (pid) {
    case 1: fill_info<1>(out); return true;
    case 3: fill_info<3>(out); return true;
    case 5: fill_info<5>(out); return true;
    default: return false;
  }
}

const void *kernel_ptr(int op, unsigned mask, int shape) {
  if (mask != 1 && mask != 2 && mask != 4) mask = 7;
  switch (op) {
    case OP_DECRYPT: return kernel_for_mask<OP_DECRYPT>(mask, shape);
    case OP_DECODE: return kernel_for_mask<OP_DECODE>(mask, shape);
    case OP_DEBUG: return kernel_for_mask<OP_DEBUG>(mask, shape);
    default: return kernel_for_mask<OP_KEYED>(mask, shape);
  }
}

size_t lds_bytes_for(int op, unsigned mask, int shape) {
  if (shape == 1) {
    if (mask == 1u) return Geo<1, 1>::LDS_BYTES;
    if (mask == 2u) return Geo<3, 1>::LDS_BYTES;
    return 0;
  }
  const bool dec = op == OP_DECODE;
  size_t b = 0;
  if (mask & 1u) b = cmax((int)b, dec ? Geo<1, 2>::LDS_BYTES : Geo<1, 0>::LDS_BYTES);
  if (mask & 2u) b = cmax((int)b, dec ? Geo<3, 2>::LDS_BYTES : Geo<3, 0>::LDS_BYTES);
  if (mask & 4u) b = cmax((int)b, dec ? Geo<5, 2>::LDS_BYTES : Geo<5, 0>::LDS_BYTES);
  return b;
}

bool shape_exists(int op, unsigned mask, int shape) {
  return kernel_ptr(op, mask, shape) != nullptr;
}

hipError_t launch(int op, unsigned mask, const KArgs &a, int grid, hipStream_t stream, int shape) {
  const void *fn = kernel_ptr(op, mask, shape);
  if (!fn) return hipErrorInvalidDeviceFunction;
  KArgs copy = a;
  void *args[] = {&copy};
  return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(64), args, lds_bytes_for(op, mask, shape),
                         stream);
}

}  // namespace hqc
