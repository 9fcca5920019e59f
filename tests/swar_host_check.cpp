// Exhaustive CPU check of the SWAR byte helpers in vbdr_device.h (saturating
// slide, fold mask, <= thr and bit-7 < c tests, nibble packing) against
// per-byte definitions.
#include "vbdr_device.h"
#include <cstdio>
using namespace vbdr;
int main() {
  long bad = 0;
  // exhaustive per-byte behaviour, bytes placed in every position with random neighbours
  unsigned seed = 1;
  auto rnd = [&]() { seed = seed * 1103515245u + 12345u; return seed >> 8; };
  for (int thr = 0; thr <= 253; ++thr) {
    uint32_t bias = swar_gt_bias(thr);
    for (int v = 0; v < 256; ++v)
      for (int pos = 0; pos < 4; ++pos)
        for (int rep = 0; rep < 4; ++rep) {
          uint32_t x = (rnd() & ~(0xFFu << (8 * pos))) | ((uint32_t)v << (8 * pos));
          uint32_t le = swar_le_mask(x, bias), inc = swar_sat_inc(x);
          for (int j = 0; j < 4; ++j) {
            uint32_t b = (x >> (8 * j)) & 0xFF;
            if (((le >> (8 * j)) & 0xFF) != (b <= (uint32_t)thr ? 0xFFu : 0u)) bad++;
            if (((inc >> (8 * j)) & 0xFF) != (b < 255 ? b + 1 : 255)) bad++;
          }
        }
  }
  // the bit-7 test below c for every c of a window k <= 128, every byte value in every position
  for (uint32_t c = 1; c <= 128; ++c) {
    const uint32_t cc = c * 0x01010101u;
    for (int v = 0; v < 256; ++v)
      for (int pos = 0; pos < 4; ++pos)
        for (int rep = 0; rep < 4; ++rep) {
          uint32_t x = (rnd() & ~(0xFFu << (8 * pos))) | ((uint32_t)v << (8 * pos));
          uint32_t lt = swar_lt_bit7(x, cc);
          for (int j = 0; j < 4; ++j) {
            uint32_t b = (x >> (8 * j)) & 0xFF;
            if (((lt >> (8 * j)) & 0xFF) != (b < c ? 0x80u : 0u)) bad++;
          }
        }
  }
  for (uint32_t f = 0; f < 16; ++f) {
    uint32_t e = swar_nibble_to_bytes(f);
    for (int j = 0; j < 4; ++j) if (((e >> (8 * j)) & 0xFF) != (((f >> j) & 1) ? 0xFFu : 0u)) bad++;
  }
  for (uint32_t a = 0; a <= 32; ++a) for (uint32_t b = 0; b <= 32; ++b) for (uint32_t c = 0; c <= 32; c += 3) for (uint32_t d = 0; d <= 32; d += 5) {
    uint32_t r = a | b << 8 | c << 16 | d << 24, n = swar_pack_nibbles(r);
    uint32_t want = (a < 15 ? a : 15) | (b < 15 ? b : 15) << 4 | (c < 15 ? c : 15) << 8 | (d < 15 ? d : 15) << 12;
    if (n != want) bad++;
  }
  printf("bad=%ld\n", bad);
  return bad != 0;
}
