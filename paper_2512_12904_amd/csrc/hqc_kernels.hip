// hqc_kernels.hip -- fused HQC.PKE.Decrypt for gfx950 (CDNA4).
//
// One workgroup = one 64-lane wavefront.  The grid is persistent: workgroup
// g handles items g, g + G, g + 2G, ... of the launch, whose items may come
// from up to three parameter sets (a public, per-item property, so the
// branch on it is uniform and data-independent).  Per item:
//
//  S0  u is staged in LDS as a bit-level doubled copy U2[t] = u[t mod n],
//      t < 2n, so every rotation of u is a contiguous window of U2.
//  S1  u*y (Eq. (1)): for support index y_k, output dword d of the product
//      is the 32 bits of U2 starting at bit 32d + n - y_k, i.e. one funnel
//      shift (v_alignbit_b32) of two adjacent U2 dwords; lane l owns the R
//      consecutive output dwords from l*R (R odd, so the 64 lanes' windows
//      hit 64 distinct LDS banks whatever the secret offset is).
//  S2  XOR with v (Alg. 2), into an LDS copy of v laid out one RM block per
//      padded row.
//  S3-S5  one RM block per lane: bit-sliced sum of the copies, 128-point
//      Walsh-Hadamard transform on packed 16-bit pairs in VGPRs, peak
//      search with smallest-index tie break, sign -> symbol byte.
//  S6-S10 Reed-Solomon with one coefficient (or position) per lane: the
//      GF(2^8) exp/log tables live in two VGPRs per lane (4 bytes each) and
//      are read with ds_bpermute_b32, a crossbar read whose timing does not
//      depend on the index; syndromes, Berlekamp-Massey in 2*delta
//      branch-free steps, error evaluator, and Chien/Forney only at the k
//      message positions (the parity positions do not reach m).
//
// Constant time: loop bounds and branches depend only on the parameter set
// and lane index; secret values flow through selects, funnel-shift amounts,
// uniform LDS window offsets and bpermute indices only.
#include "hqc_internal.h"

namespace hqc {
namespace {

// ---- parameter sets (Table I) --------------------------------------------
template <int ID> struct Set;
template <> struct Set<1> { static constexpr int n = 17669, n1 = 46, n2 = 384, k = 16, delta = 15, w = 66; };
template <> struct Set<3> { static constexpr int n = 35851, n1 = 56, n2 = 640, k = 24, delta = 16, w = 100; };
template <> struct Set<5> { static constexpr int n = 57637, n1 = 90, n2 = 640, k = 32, delta = 29, w = 131; };

template <int ID> struct Geo {
  using S = Set<ID>;
  static constexpr int n = S::n, n1 = S::n1, n2 = S::n2, k = S::k, w = S::w;
  static constexpr int MULT = n2 / 128;
  static constexpr int TD = 2 * S::delta;            // number of syndromes
  static constexpr int W32 = n1 * n2 / 32;           // dwords of v and of the product we keep
  static constexpr int R = ((W32 + 63) / 64) | 1;    // product dwords per lane (odd)
  static constexpr int DW = n / 32;                  // dword holding bit n - 1
  static constexpr int NB = n % 32;                  // bits of u in dword DW
  static constexpr int U_WORDS = (n + 63) / 64;
  static constexpr int V_WORDS = n1 * n2 / 64;
  static constexpr int BLK = 4 * MULT;               // dwords per RM block
  static constexpr int BSTR = BLK + 1;               // padded LDS row of a block
  static constexpr int U2 = 64 * R + DW + 2;         // doubled-u dwords (covers every window)
  static constexpr int RB = n1 * BSTR;               // received-word dwords
  static constexpr int LDS = U2 + RB;                // LDS dwords per workgroup
  static constexpr int YREG = (w + 63) / 64;         // VGPRs holding y
  static constexpr int SYMREG = (n1 + 63) / 64;      // VGPRs holding the symbols
  static_assert(NB != 0, "n is not a multiple of 32 for any HQC set");
  static_assert(TD + 1 <= 64 && k <= 64, "one lane per RS coefficient / message byte");
  static_assert(n1 * n2 % 64 == 0, "v is a whole number of words");
  static_assert(64 * R >= W32, "lanes cover the product");
};

// ---- GF(2^8) tables, x^8 + x^4 + x^3 + x^2 + 1, alpha = x ------------------
struct GfTables {
  uint32_t exp4[64];  // bytes exp[4l .. 4l+3]; exp[255] = exp[0] = 1
  uint32_t log4[64];  // bytes log[4l .. 4l+3]; log[0] = 0 (callers mask zero)
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
  e[255] = 1;  // lets a log sum in [0, 510] be reduced by (s + (s >> 8)) & 255
  for (int i = 0; i < 64; ++i) {
    t.exp4[i] = (uint32_t)e[4 * i] | (uint32_t)e[4 * i + 1] << 8 | (uint32_t)e[4 * i + 2] << 16 |
                (uint32_t)e[4 * i + 3] << 24;
    t.log4[i] = (uint32_t)l[4 * i] | (uint32_t)l[4 * i + 1] << 8 | (uint32_t)l[4 * i + 2] << 16 |
                (uint32_t)l[4 * i + 3] << 24;
  }
  return t;
}

__constant__ GfTables kGf = make_gf_tables();

typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x; }

// Table read: byte idx (0..255) of a table spread over the wave, 4 bytes per
// lane.  Must run with all 64 lanes active.
__device__ __forceinline__ uint32_t tab(uint32_t table4, uint32_t idx) {
  uint32_t w = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(idx & 0xFCu), (int)table4);
  return __builtin_amdgcn_ubfe(w, (idx & 3u) << 3, 8);
}

// (s mod 255) for s in [0, 510], as an exp-table index (255 stands for 0)
__device__ __forceinline__ uint32_t mod255(uint32_t s) { return (s + (s >> 8)) & 0xFFu; }

__device__ __forceinline__ uint32_t wave_xor(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v ^= (uint32_t)__shfl_xor((int)v, o);
  return v;
}

__device__ __forceinline__ uint32_t rdlane(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

__device__ __forceinline__ uint32_t from_lane(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)v);
}

// ---- S3-S5: one duplicated RM(1,7) block -> symbol byte ---------------------
template <int MULT>
__device__ __forceinline__ uint32_t rm_decode_block(const uint32_t *blk) {
  // bit-sliced count of set copies per position: F = p0 + 2 p1 + 4 p2
  uint32_t p0[4], p1[4], p2[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t a = blk[q], b = blk[4 + q], c = blk[8 + q];
    uint32_t s = a ^ b ^ c, cy = (a & b) | (c & (a ^ b));
    if constexpr (MULT == 3) {
      p0[q] = s;
      p1[q] = cy;
      p2[q] = 0;
    } else {
      uint32_t d = blk[12 + q], e = blk[16 + q];
      uint32_t s2 = s ^ d ^ e, cy2 = (s & d) | (e & (s ^ d));
      p0[q] = s2;
      p1[q] = cy ^ cy2;
      p2[q] = cy & cy2;
    }
  }
  // packed pairs (2m, 2m+1) after the first transform stage
  s16x2 h[64];
#pragma unroll
  for (int m = 0; m < 64; ++m) {
    const int q = m >> 4, b = (2 * m) & 31;
    int f0 = (int)(((p0[q] >> b) & 1u) + 2u * ((p1[q] >> b) & 1u) + 4u * ((p2[q] >> b) & 1u));
    int f1 = (int)(((p0[q] >> (b + 1)) & 1u) + 2u * ((p1[q] >> (b + 1)) & 1u) +
                   4u * ((p2[q] >> (b + 1)) & 1u));
    h[m] = s16x2{(short)(f0 + f1), (short)(f0 - f1)};
  }
#pragma unroll
  for (int hh = 1; hh < 64; hh <<= 1) {
#pragma unroll
    for (int m = 0; m < 64; ++m) {
      if (m & hh) continue;
      s16x2 a = h[m], c = h[m + hh];
      h[m] = a + c;
      h[m + hh] = a - c;
    }
  }
  // H = transform of the counts; the correlation with codeword (u, sign) is
  // T(u) = 128*MULT*[u == 0] - 2 H(u) = -2 H'(u), H'(0) = H(0) - 64*MULT.
  h[0].x = (short)(h[0].x - 64 * MULT);
  uint32_t best = 0;
#pragma unroll
  for (int m = 0; m < 64; ++m) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int u = 2 * m + half;
      int v = half ? h[m].y : h[m].x;
      uint32_t mag = (uint32_t)(v < 0 ? -v : v);
      uint32_t key = (mag << 8) | (uint32_t)((127 - u) << 1) | (v > 0 ? 1u : 0u);
      best = best > key ? best : key;
    }
  }
  uint32_t ustar = 127u - ((best >> 1) & 127u);
  return ustar | ((best & 1u) << 7);  // T(u*) < 0  <=>  H'(u*) > 0
}

// ---- one item ----------------------------------------------------------------
template <int ID, int OP>
__device__ __forceinline__ void run_item(const SegDev &sg, uint32_t item, uint32_t *lds,
                                         uint32_t exp4, uint32_t log4) {
  using G = Geo<ID>;
  const int lane = (int)lane_id();
  uint32_t *u2 = lds;
  uint32_t *rb = lds + G::U2;

  // key slot (keyed): ids are device data; out-of-range ids decrypt to zeros
  uint32_t key = 0;
  bool bad_key = false;
  if constexpr (OP == OP_KEYED) {
    key = __builtin_amdgcn_readfirstlane(sg.key_ids[item]);
    bad_key = key >= sg.ks_cap;
    key = bad_key ? 0u : key;
  }

  // S2 input: v (decrypt) or r (decode), one padded row per RM block
  const uint32_t *vsrc = (const uint32_t *)((OP == OP_DECODE ? sg.u : sg.v) +
                                            (size_t)item * G::V_WORDS);
  for (int d = lane; d < G::W32; d += 64) rb[d + d / G::BLK] = vsrc[d];

  if constexpr (OP != OP_DECODE) {
    // S0: U2[0 .. DW) = u, then U2[DW ..] = the wrapped continuation
    const uint32_t *usrc = (const uint32_t *)(sg.u + (size_t)item * G::U_WORDS);
    for (int d = lane; d < G::DW; d += 64) u2[d] = usrc[d];
    const uint32_t udw = __builtin_amdgcn_readfirstlane(usrc[G::DW]) & ((1u << G::NB) - 1u);
    const uint32_t *ysrc = (OP == OP_KEYED) ? sg.ks_y + (size_t)key * G::w : sg.y + (size_t)item * G::w;
    uint32_t yreg[G::YREG];
#pragma unroll
    for (int c = 0; c < G::YREG; ++c) {
      int idx = 64 * c + lane;
      yreg[c] = idx < G::w ? ysrc[idx] : 0u;
    }
    __syncthreads();
    for (int D = G::DW + lane; D < G::U2; D += 64) {
      const int i = D - G::DW;  // >= 0
      uint32_t val;
      if (i == 0) {
        val = udw | (u2[0] << G::NB);
      } else {
        const int ih = i < G::DW ? i : G::DW - 1, il = i - 1 < G::DW ? i - 1 : G::DW - 1;
        uint32_t hi = i < G::DW ? u2[ih] : (i == G::DW ? udw : 0u);
        uint32_t lo = i - 1 < G::DW ? u2[il] : (i - 1 == G::DW ? udw : 0u);
        val = __builtin_amdgcn_alignbit(hi, lo, 32 - G::NB);
      }
      u2[D] = val;
    }
    __syncthreads();

    // S1: product, R output dwords per lane
    uint32_t acc[G::R];
#pragma unroll
    for (int j = 0; j < G::R; ++j) acc[j] = 0;
    const uint32_t *base = u2 + lane * G::R;
#pragma unroll
    for (int c = 0; c < G::YREG; ++c) {
      const int cnt = (G::w - 64 * c) < 64 ? (G::w - 64 * c) : 64;
      for (int kk = 0; kk < cnt; ++kk) {
        uint32_t yk = rdlane(yreg[c], kk) % (uint32_t)G::n;
        uint32_t sh = (uint32_t)G::n - yk;  // in [1, n]
        const uint32_t *p = base + (sh >> 5);
        const uint32_t s = sh & 31u;
        uint32_t win[G::R + 1];
#pragma unroll
        for (int j = 0; j <= G::R; ++j) win[j] = p[j];
#pragma unroll
        for (int j = 0; j < G::R; ++j) acc[j] ^= __builtin_amdgcn_alignbit(win[j + 1], win[j], s);
      }
    }
    // S2: r = v + (u*y) restricted to the first n1*n2 bits
#pragma unroll
    for (int j = 0; j < G::R; ++j) {
      const int d = lane * G::R + j;
      if (d < G::W32) rb[d + d / G::BLK] ^= acc[j];
    }
  }
  __syncthreads();

  // S3-S5: RM blocks, one per lane
  uint32_t sym[G::SYMREG];
#pragma unroll
  for (int pass = 0; pass < G::SYMREG; ++pass) {
    int j = lane + 64 * pass;
    int jj = j < G::n1 ? j : G::n1 - 1;
    sym[pass] = rm_decode_block<G::MULT>(rb + jj * G::BSTR);
  }

  // S6: syndromes, lane i holds S_i (i = 1 .. TD)
  uint32_t logc[G::SYMREG];
#pragma unroll
  for (int pass = 0; pass < G::SYMREG; ++pass) logc[pass] = tab(log4, sym[pass]);
  uint32_t S = 0, ij = 0;
  const uint32_t il = (uint32_t)lane;
#pragma unroll
  for (int pass = 0; pass < G::SYMREG; ++pass) {
    const int cnt = (G::n1 - 64 * pass) < 64 ? (G::n1 - 64 * pass) : 64;
    for (int j = 0; j < cnt; ++j) {
      uint32_t lc = rdlane(logc[pass], j);
      uint32_t cz = rdlane(sym[pass], j);
      uint32_t t = tab(exp4, mod255(lc + ij));
      S ^= cz ? t : 0u;
      ij += il;
      ij = ij >= 255u ? ij - 255u : ij;
    }
  }
  S = (lane >= 1 && lane <= G::TD) ? S : 0u;

  // S7: Berlekamp-Massey with B' = x^s B / b (lane i holds coefficient i)
  const uint32_t logS = tab(log4, S) | (S == 0 ? 0x100u : 0u);
  uint32_t lam = lane == 0 ? 1u : 0u;
  uint32_t bb = lane == 1 ? 1u : 0u;
  int L = 0;
  for (int r = 1; r <= G::TD; ++r) {
    const int src = r - lane;
    const bool valid = src >= 1;
    const uint32_t lS = from_lane(logS, valid ? src : 0);
    const uint32_t lL = tab(log4, lam);
    uint32_t term = tab(exp4, mod255(lL + (lS & 0xFFu)));
    term = (valid && lam != 0 && !(lS & 0x100u)) ? term : 0u;
    const uint32_t delta = __builtin_amdgcn_readfirstlane(wave_xor(term));
    const uint32_t lD = tab(log4, delta);
    const bool nz = delta != 0;
    const uint32_t lB = tab(log4, bb);
    uint32_t t1 = tab(exp4, mod255(lD + lB));
    t1 = (nz && bb != 0) ? t1 : 0u;
    uint32_t q = tab(exp4, mod255(lL + 255u - lD));
    q = (nz && lam != 0) ? q : 0u;
    const bool swap = nz && (2 * L <= r - 1);
    const uint32_t pre = swap ? q : bb;
    const uint32_t up = from_lane(pre, lane > 0 ? lane - 1 : 0);
    bb = (lane >= 1 && lane <= G::TD) ? up : 0u;
    lam = lane <= G::TD ? (lam ^ t1) : 0u;
    L = swap ? r - L : L;
  }

  // S9 (part): Omega = S(x) Lambda(x) mod x^TD, lane e holds Omega_e
  const uint32_t lLam = tab(log4, lam);
  uint32_t om = 0;
  for (int i = 0; i <= G::TD; ++i) {
    const uint32_t li = rdlane(lLam, i);
    const uint32_t zi = rdlane(lam, i);
    const int src = lane + 1 - i;
    const bool valid = src >= 1 && src <= G::TD;
    const uint32_t lS = from_lane(logS, valid ? src : 0);
    uint32_t t = tab(exp4, mod255(li + (lS & 0xFFu)));
    om ^= (valid && zi != 0 && !(lS & 0x100u)) ? t : 0u;
  }
  om = lane < G::TD ? om : 0u;

  // S8-S10: Chien + Forney at message position j = TD + lane
  const uint32_t lOm = tab(log4, om);
  const uint32_t jm = (uint32_t)(G::TD + (lane < G::k ? lane : 0));  // < 255
  uint32_t ex = 0;  // (-i j) mod 255
  uint32_t lamv = 0, oddv = 0, omv = 0;
  for (int i = 0; i <= G::TD; ++i) {
    const uint32_t li = rdlane(lLam, i), zi = rdlane(lam, i);
    uint32_t t = tab(exp4, mod255(li + ex));
    t = zi ? t : 0u;
    lamv ^= t;
    oddv ^= (i & 1) ? t : 0u;
    if (i < G::TD) {
      const uint32_t lo = rdlane(lOm, i), zo = rdlane(om, i);
      uint32_t t2 = tab(exp4, mod255(lo + ex));
      omv ^= zo ? t2 : 0u;
    }
    ex = ex >= jm ? ex - jm : ex + 255u - jm;
  }
  // e_j = Omega(X^-1) / Lambda'(X^-1), Lambda'(X^-1) = X * odd part of Lambda at X^-1
  const uint32_t l1 = mod255(tab(log4, omv) + 255u - tab(log4, oddv));
  uint32_t e = tab(exp4, mod255(l1 + 255u - jm));
  e = (lamv == 0 && omv != 0 && oddv != 0) ? e : 0u;
  const int j = G::TD + lane;
  uint32_t cj = from_lane(sym[0], j < 64 ? j : 0);
  if constexpr (G::SYMREG > 1) {
    const uint32_t c1 = from_lane(sym[G::SYMREG - 1], j >= 64 ? j - 64 : 0);
    cj = j >= 64 ? c1 : cj;
  }
  uint32_t mbyte = (cj ^ e) & 0xFFu;
  if constexpr (OP == OP_KEYED) mbyte = bad_key ? 0u : mbyte;
  if (lane < G::k) sg.m[(size_t)item * G::k + lane] = (uint8_t)mbyte;
  if constexpr (OP == OP_KEYED) {
    if (bad_key && lane == 0) atomicAdd(sg.ks_bad, 1ull);
  }
  __syncthreads();
}

template <int OP, unsigned MASK>
__global__ __launch_bounds__(64) void hqc_kernel(KArgs a) {
  extern __shared__ uint32_t lds[];
  const uint32_t exp4 = kGf.exp4[lane_id()];
  const uint32_t log4 = kGf.log4[lane_id()];
  for (uint32_t unit = blockIdx.x; unit < a.total; unit += gridDim.x) {
    int s = 0;
    if (a.nseg > 1 && unit >= a.seg[1].first) s = 1;
    if (a.nseg > 2 && unit >= a.seg[2].first) s = 2;
    const SegDev &sg = a.seg[s];
    const uint32_t item = unit - sg.first;
    if ((MASK & 1u) && sg.pid == 1) run_item<1, OP>(sg, item, lds, exp4, log4);
    if ((MASK & 2u) && sg.pid == 3) run_item<3, OP>(sg, item, lds, exp4, log4);
    if ((MASK & 4u) && sg.pid == 5) run_item<5, OP>(sg, item, lds, exp4, log4);
  }
}

template <int OP>
const void *kernel_for_mask(unsigned mask) {
  switch (mask) {
    case 1: return (const void *)&hqc_kernel<OP, 1>;
    case 2: return (const void *)&hqc_kernel<OP, 2>;
    case 4: return (const void *)&hqc_kernel<OP, 4>;
    default: return (const void *)&hqc_kernel<OP, 7>;
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
  o->lds_bytes = sizeof(uint32_t) * G::LDS;
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

const void *kernel_ptr(int op, unsigned mask) {
  if (mask != 1 && mask != 2 && mask != 4) mask = 7;
  switch (op) {
    case OP_DECRYPT: return kernel_for_mask<OP_DECRYPT>(mask);
    case OP_DECODE: return kernel_for_mask<OP_DECODE>(mask);
    default: return kernel_for_mask<OP_KEYED>(mask);
  }
}

size_t lds_bytes_for(unsigned mask) {
  size_t b = 0;
  SetInfo si;
  if (mask & 1u) { set_info(1, &si); b = si.lds_bytes > b ? si.lds_bytes : b; }
  if (mask & 2u) { set_info(3, &si); b = si.lds_bytes > b ? si.lds_bytes : b; }
  if (mask & 4u) { set_info(5, &si); b = si.lds_bytes > b ? si.lds_bytes : b; }
  return b;
}

hipError_t launch(int op, unsigned mask, const KArgs &a, int grid, hipStream_t stream) {
  const void *fn = kernel_ptr(op, mask);
  KArgs copy = a;
  void *args[] = {&copy};
  return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(64), args, lds_bytes_for(mask), stream);
}

}  // namespace hqc
