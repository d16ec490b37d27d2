// Host-side check of the GPU kernels' index arithmetic (built host-only by
// tests/test_bounds_model.py; no GPU needed).  It evaluates the index
// functions the kernels themselves call (Layout<G> in hqc_device.h) for every
// geometry the library instantiates -- HQC-1/3/5 in shape 0 and in the
// decoding layout, HQC-1/3 in shape 1 -- over every lane, every shift of the
// product windows, every tile size and every RM pass of the pass schedule,
// and checks each LDS
// offset against the layout's region and the dynamic LDS size, and each row
// offset against the row sizes of the device buffers.  Prints one line per
// geometry and exits non-zero on the first violation.
#include <cstdint>
#include <cstdio>
#include <cstdlib>

#include "hqc_device.h"

namespace {

int failures = 0;

void fail(const char *geo, const char *what, long a, long b) {
  if (failures++ < 20) std::printf("FAIL %s: %s (%ld vs %ld)\n", geo, what, a, b);
}

#define CHECK(geo, cond, what, a, b) \
  do {                               \
    if (!(cond)) fail(geo, what, (long)(a), (long)(b)); \
  } while (0)

template <int ID, int SH> void check_decrypt(const char *name) {
  using G = hqc::Geo<ID, SH>;
  using L = hqc::Layout<G>;
  const long lds_dw = G::LDS_BYTES / 4, a_dw = G::A_BYTES / 4;
  CHECK(name, G::LDS_BYTES % 4 == 0 && G::A_BYTES % 16 == 0, "alignment", G::LDS_BYTES, G::A_BYTES);
  CHECK(name, G::LDS_BYTES * 4 * G::WAVES <= 160 * 1024, "LDS of the resident wavefronts",
        G::LDS_BYTES * 4 * G::WAVES, 160 * 1024);
  // S0: the doubled copy (written for D < U2) lies in the first region --
  // except in the decoding layout, which has none
  if constexpr (!G::DECODE_ONLY) {
    CHECK(name, G::U2 <= a_dw, "doubled copy inside the received-word region", G::U2, a_dw);
    CHECK(name, G::COMPACT || L::rb(0) >= G::U2, "rows after the doubled copy", L::rb(0), G::U2);
    // S1: every product window dword, every lane, every shift in [1, n]
    for (int lane = 0; lane < 64; ++lane)
      for (uint32_t sh = 1; sh <= (uint32_t)G::n; ++sh) {
        const int lo = L::window(lane, sh, 0), hi = L::window(lane, sh, G::R);
        CHECK(name, lo >= 0 && hi < G::U2, "product window inside the doubled copy", hi, G::U2);
      }
  }
  // S2: received-word rows of every slot
  for (int q = 0; q < G::RMG; ++q) {
    for (int d = 0; d < G::W32; ++d) {
      const int o = L::rb(q) + L::row(d);
      CHECK(name, o >= L::rb(q) && o < L::rb(q) + G::RB, "row inside its slot", o, L::rb(q) + G::RB);
      CHECK(name, o < a_dw, "row inside the region", o, a_dw);
    }
    if constexpr (!G::DECODE_ONLY)
      for (int lane = 0; lane < 64; ++lane)
        for (int j = 0; j < G::R; ++j) {
          const int d = L::out(lane, j);
          if (d < G::W32) CHECK(name, L::rb(q) + L::row(d) < a_dw, "product row", d, a_dw);
        }
  }
  // S3-S5: the RM pass schedule for every tile size, and the symbol stores
  for (int nt = 1; nt <= G::TROWS; ++nt) {
    int passes = 0;
    for (int it = 0; it < nt; ++it) {
      const int gi = it % G::RMG;
      const int g0 = it - gi, avail = (gi + 1) * G::n1;
      const bool last = gi == G::RMG - 1 || it == nt - 1;
      if (gi == 0) passes = 0;
      while (passes * L::BPP < avail && ((passes + 1) * L::BPP <= avail || last)) {
        for (int lane = 0; lane < 64; ++lane) {
          const int fl = L::pass_flat(passes, lane);
          const int f = L::pass_clamp(fl, avail);
          const int q = f / G::n1, b = f - q * G::n1;
          CHECK(name, f >= 0 && q <= gi, "block of a received word", q, gi);
          const int blk = L::block(q, b);
          CHECK(name, blk >= L::rb(q) && blk + G::BLK - 1 < L::rb(q) + G::RB, "block inside its slot",
                blk + G::BLK, L::rb(q) + G::RB);
          if (fl < avail && lane < L::BPP) {
            CHECK(name, g0 + q < nt && b < G::n1, "symbol of a tile row", g0 + q, nt);
            // rows follow the pending rows of earlier tiles: a piece of at
            // most 32 items starts at any row0 with row0 + nt <= 32, a larger
            // one at row 0
            const int row0_max = nt <= 32 ? 32 - nt : 0;
            for (int row0 = 0; row0 <= row0_max; row0 += row0_max > 0 ? row0_max : 1) {
              const int so = L::sym(row0 + g0 + q, b);
              CHECK(name, row0 + g0 + q < G::TROWS, "symbol row inside the table", row0 + g0 + q,
                    G::TROWS);
              CHECK(name, so >= G::A_BYTES && so < G::LDS_BYTES, "symbol store inside the table",
                    so, G::LDS_BYTES);
            }
          }
        }
        ++passes;
      }
      if (last) CHECK(name, passes * L::BPP >= avail, "every block of the group decoded", passes, avail);
    }
    // S6-S10: each lane (or lane pair) reads one pending row's symbols
    // (nt rows pending; at most 32 for the pair form, up to TROWS otherwise)
    const bool pair = G::COMPACT || nt <= 32;
    for (int lane = 0; lane < 64; ++lane) {
      const int s = pair ? (lane & 31) : lane;
      const int slot = s < nt ? s : 0;
      CHECK(name, L::sym(slot, 0) >= G::A_BYTES && L::sym(slot, G::n1 - 1) < G::LDS_BYTES,
            "symbol row read", L::sym(slot, G::n1 - 1), G::LDS_BYTES);
    }
  }
  // device rows: u (u_words words), v / r (v_words), y (w), m (k bytes, dwords)
  CHECK(name, G::DW < 2 * G::U_WORDS, "u dwords read", G::DW, 2 * G::U_WORDS);
  CHECK(name, G::W32 <= 2 * G::V_WORDS, "v dwords read", G::W32, 2 * G::V_WORDS);
  CHECK(name, G::k % 4 == 0, "m written a dword at a time", G::k, 4);
  CHECK(name, G::DBG_E + G::k <= G::DBG_BYTES && G::DBG_BYTES % 4 == 0, "debug record",
        G::DBG_E + G::k, G::DBG_BYTES);
  (void)lds_dw;
}

template <int ID> void check_encrypt(const char *name) {
  using G = hqc::Geo<ID>;
  using L = hqc::Layout<G>;
  // staging buffer (dwords 0 .. DW written, W32 for v) inside the doubled copy
  for (int lane = 0; lane < 64; ++lane)
    for (int j = 0; j < G::R; ++j) {
      const int d = L::out(lane, j);
      if (d <= G::DW) CHECK(name, d < G::U2, "staging dword", d, G::U2);
    }
  CHECK(name, G::W32 <= G::U2, "v staging", G::W32, G::U2);
  // sparse additions: dword q / 32 for every index q < n
  CHECK(name, (G::n - 1) >> 5 == G::DW && G::DW < G::U2, "sparse addition dword", G::DW, G::U2);
  // symbol table after the doubled copy: parity (lanes < 2 delta), message
  // (2 delta + lanes < k), the codeword symbols read back (< n1)
  CHECK(name, L::enc_sym(0) == 4 * G::U2, "symbol table start", L::enc_sym(0), 4 * G::U2);
  CHECK(name, L::enc_sym(G::TD + G::k - 1) < L::ENC_LDS_BYTES && L::enc_sym(G::n1 - 1) < L::ENC_LDS_BYTES,
        "symbol table end", L::enc_sym(G::n1 - 1), L::ENC_LDS_BYTES);
  for (int lane = 0; lane < 64; ++lane)
    for (uint32_t sh = 1; sh <= (uint32_t)G::n; sh += 1 + (sh & 7))
      CHECK(name, L::window(lane, sh, G::R) < G::U2, "window", L::window(lane, sh, G::R), G::U2);
}

}  // namespace

// The tile schedule of a launch over several segments: every tile is taken
// by exactly one workgroup, inside its own segment, and its items lie inside
// the segment.
void check_schedule() {
  const char *name = "tile schedule";
  const uint32_t counts[][3] = {{1, 0, 0}, {64, 65, 1}, {0, 100, 7}, {1000, 999, 998},
                                {32768, 19661, 13107}, {5, 0, 130}};
  const uint32_t tiles[][3] = {{1, 1, 1}, {64, 30, 16}, {7, 3, 2}, {32, 15, 8}};
  const uint32_t grids[] = {1, 3, 64, 2048, 3072};
  for (const auto &c : counts)
    for (const auto &t : tiles)
      for (uint32_t grid : grids) {
        uint32_t first[4], total = 0;
        for (int s = 0; s < 3; ++s) {
          first[s] = total;
          total += (c[s] + t[s] - 1) / t[s];
        }
        first[3] = total;
        if (grid > total && total > 0) grid = total;
        if (total == 0) continue;
        static unsigned char seen[1 << 20];
        for (uint32_t u = 0; u < total; ++u) seen[u] = 0;
        for (uint32_t b = 0; b < grid; ++b)
          for (int s = 0; s < 3; ++s)
            for (uint32_t u = hqc::first_unit(b, grid, first[s]); u < first[s + 1]; u += grid) {
              CHECK(name, u % grid == b, "tile of another workgroup", u, b);
              CHECK(name, u >= first[s], "tile before its segment", u, first[s]);
              ++seen[u];
              const uint32_t item0 = (u - first[s]) * t[s];
              const uint32_t nt = c[s] - item0 < t[s] ? c[s] - item0 : t[s];
              CHECK(name, item0 < c[s] && nt >= 1 && item0 + nt <= c[s], "items inside the segment",
                    item0 + nt, c[s]);
            }
        for (uint32_t u = 0; u < total; ++u) CHECK(name, seen[u] == 1, "tile taken once", u, seen[u]);
      }
}

int main() {
  check_schedule();
  std::printf("tile schedule ok\n");
  check_decrypt<1, 0>("decrypt HQC-1 shape A");
  std::printf("decrypt HQC-1 shape A ok\n");
  check_decrypt<1, 1>("decrypt HQC-1 shape B");
  std::printf("decrypt HQC-1 shape B ok\n");
  check_decrypt<3, 0>("decrypt HQC-3 shape A");
  std::printf("decrypt HQC-3 shape A ok\n");
  check_decrypt<3, 1>("decrypt HQC-3 shape B");
  std::printf("decrypt HQC-3 shape B ok\n");
  check_decrypt<5, 0>("decrypt HQC-5");
  std::printf("decrypt HQC-5 ok\n");
  check_decrypt<1, 2>("decode HQC-1");
  check_decrypt<3, 2>("decode HQC-3");
  check_decrypt<5, 2>("decode HQC-5");
  std::printf("decoding layouts ok\n");
  check_encrypt<1>("encrypt HQC-1");
  check_encrypt<3>("encrypt HQC-3");
  check_encrypt<5>("encrypt HQC-5");
  std::printf("encrypt ok\n");
  if (failures) std::printf("%d violations\n", failures);
  return failures ? 1 : 0;
}
