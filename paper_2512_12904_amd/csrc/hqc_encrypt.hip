// hqc_encrypt.hip -- batched HQC key generation (Alg. 3: s = x + h*y) and
// PKE encryption (Alg. 1: u = r1 + h*r2, v = mG + s*r2 + e truncated to
// n1*n2 bits) for gfx950.  The randomness (h, x, y, r1, r2, e, m) is an
// input; nothing here draws random numbers.
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

// a*(support) + 1*(support2) -> acc (all R dwords of every lane)
template <int ID, int N1, int N2>
__device__ __forceinline__ void two_products(const uint32_t *u2, const uint32_t *one,
                                             const uint32_t *supp1, const uint32_t *supp2,
                                             uint32_t (&acc)[Geo<ID>::R]) {
  uint32_t i1[(N1 + 63) / 64], s1[(N1 + 63) / 64], i2[(N2 + 63) / 64], s2[(N2 + 63) / 64];
  load_support<N1>(supp1, i1);
  load_support<N2>(supp2, i2);
  window_shifts<ID, (N1 + 63) / 64>(i1, s1);
  window_shifts<ID, (N2 + 63) / 64>(i2, s2);
#pragma unroll
  for (int j = 0; j < Geo<ID>::R; ++j) acc[j] = 0;
  product_acc<ID, N1>(u2, s1, acc);
  product_acc<ID, N2>(one, s2, acc);
}

// store a full n-bit polynomial (bits >= n cleared) from the lanes' dwords
template <int ID>
__device__ __forceinline__ void store_full(uint64_t *row, const uint32_t (&acc)[Geo<ID>::R]) {
  using G = Geo<ID>;
  uint32_t *dst = (uint32_t *)row;
  const int lane = lane_id();
#pragma unroll
  for (int j = 0; j < G::R; ++j) {
    const int d = lane * G::R + j;
    if (d < 2 * G::U_WORDS) {
      uint32_t val = d < G::DW ? acc[j] : (d == G::DW ? acc[j] & ((1u << G::NB) - 1u) : 0u);
      dst[d] = val;
    }
  }
}

template <int ID, bool ENCRYPT>
__device__ __forceinline__ void run_item(const EncArgs &a, uint32_t item, uint32_t *lds,
                                         uint32_t exp4, uint32_t log4, uint32_t pat) {
  using G = Geo<ID>;
  const int lane = lane_id();
  uint32_t *u2 = lds;
  uint32_t *one = lds + G::U2;
  uint8_t *sym = (uint8_t *)(lds + 2 * G::U2);
  uint32_t acc[G::R];
  const size_t nw = (size_t)G::U_WORDS;

  if constexpr (!ENCRYPT) {
    // Alg. 3: s = x + h*y
    stage_dense<ID>(a.h + item * nw, u2);
    two_products<ID, G::w, G::w>(u2, one, a.y + (size_t)item * G::w, a.x + (size_t)item * G::w, acc);
    store_full<ID>(a.s_out + item * nw, acc);
    wave_sync();
    return;
  } else {
    constexpr int WR = Set<ID>::wr;
    // Alg. 1: u = r1 + h*r2
    stage_dense<ID>(a.h + item * nw, u2);
    two_products<ID, WR, WR>(u2, one, a.r2 + (size_t)item * WR, a.r1 + (size_t)item * WR, acc);
    store_full<ID>(a.u_out + item * nw, acc);

    // Reed-Solomon parity of m: x^{2d} m(x) mod g(x), register j in lane j
    constexpr int TD = G::TD;
    const uint8_t *mrow = a.m + (size_t)item * G::k;
    const uint32_t lg = kRsGen.lg[gen_slot<ID>()][lane];
    const uint32_t gnz = kRsGen.nz[gen_slot<ID>()][lane];
    uint32_t reg = 0;
#pragma unroll 1
    for (int t = G::k - 1; t >= 0; --t) {
      const uint32_t mt = __builtin_amdgcn_readfirstlane((uint32_t)mrow[t]);
      const uint32_t fb = (mt ^ rdlane(reg, TD - 1)) & 0xFFu;
      const uint32_t lfb = tab(log4, fb);
      uint32_t prod = tab(exp4, red255(lfb + lg));
      prod = (fb != 0 && gnz) ? prod : 0u;
      const uint32_t prev = (uint32_t)__builtin_amdgcn_ds_bpermute((lane > 0 ? lane - 1 : 0) << 2,
                                                                  (int)reg);
      reg = lane < TD ? ((lane > 0 ? prev : 0u) ^ prod) : 0u;
    }
    if (lane < TD) sym[lane] = (uint8_t)reg;
    if (lane < G::k) sym[TD + lane] = mrow[lane];

    // v = mG + s*r2 + e, first n1*n2 bits
    wave_sync();
    stage_dense<ID>(a.s + item * nw, u2);
    two_products<ID, WR, Set<ID>::we>(u2, one, a.r2 + (size_t)item * WR,
                                      a.e + (size_t)item * Set<ID>::we, acc);
    uint32_t *dst = (uint32_t *)(a.v_out + item * (size_t)G::V_WORDS);
#pragma unroll
    for (int j = 0; j < G::R; ++j) {
      const int d = lane * G::R + j;
      const int dd = d < G::W32 ? d : 0;
      const int blk = dd / G::BLK, w = (dd % G::BLK) & 3;
      const uint32_t c = sym[blk];
      const uint32_t p = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((c & 31u) << 2), (int)pat);
      const uint32_t flip = ((c >> 7) ^ ((c >> 5) & (uint32_t)w) ^ ((c >> 6) & ((uint32_t)w >> 1))) & 1u;
      const uint32_t word = p ^ (0u - flip);
      if (d < G::W32) dst[d] = acc[j] ^ word;
    }
    wave_sync();
  }
}

template <bool ENCRYPT, int ID>
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
    run_item<ID, ENCRYPT>(a, item, lds, exp4, log4, pat);
}

template <int ID> size_t enc_lds() {
  using G = Geo<ID>;
  return sizeof(uint32_t) * 2 * G::U2 + ((G::n1 + 63) / 64) * 64;
}

}  // namespace

const void *encrypt_kernel_ptr(bool encrypt, int pid) {
  if (encrypt) {
    switch (pid) {
      case 1: return (const void *)&hqc_encrypt_kernel<true, 1>;
      case 3: return (const void *)&hqc_encrypt_kernel<true, 3>;
      default: return (const void *)&hqc_encrypt_kernel<true, 5>;
    }
  }
  switch (pid) {
    case 1: return (const void *)&hqc_encrypt_kernel<false, 1>;
    case 3: return (const void *)&hqc_encrypt_kernel<false, 3>;
    default: return (const void *)&hqc_encrypt_kernel<false, 5>;
  }
}

size_t encrypt_lds_bytes(int pid) {
  switch (pid) {
    case 1: return enc_lds<1>();
    case 3: return enc_lds<3>();
    default: return enc_lds<5>();
  }
}

hipError_t launch_encrypt(bool encrypt, int pid, const EncArgs &a, int grid, hipStream_t stream) {
  EncArgs copy = a;
  void *args[] = {&copy};
  return hipLaunchKernel(encrypt_kernel_ptr(encrypt, pid), dim3((unsigned)grid), dim3(64), args,
                         encrypt_lds_bytes(pid), stream);
}

}  // namespace hqc
