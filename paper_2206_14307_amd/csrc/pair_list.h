// Second-hop bond list of the two-hop kernels (H^2 terms, Sec. 3.3).
#pragma once
#include <cstdint>

#include "device_common.h"

namespace nqs {

constexpr int kPairTwice = 0x4000;   // list flag: the unordered pair counts twice
constexpr int kPairBond = 0x3fff;    // list mask: the bond index

// For first hop b1 = (i1, j1) of configuration s, with row2 = s^{b1}: the
// antiparallel bonds b2 of s^{b1} except b1 itself (exchanging it back
// returns s: the kernels add that term, (J_b1/2)^2 per unit image weight, in
// closed form), and of the bonds sharing no site with b1 only those with
// b2 > b1.  Disjoint exchanges commute, so s^{b1 b2} = s^{b2 b1} with the
// same weight (J_b1 J_b2 / 4): such an entry carries the flag 0x4000 and
// counts twice.  Returns the list length; one wavefront, list in LDS.
__device__ __forceinline__ int build_pair_list(const int8_t* row2, const int32_t* bonds, int NB,
                                               int16_t* list, int lane, int b1, int i1, int j1) {
  int n = 0;
  for (int base = 0; base < NB; base += 64) {
    const int b = base + lane;
    bool keep = false, twice = false;
    if (b < NB && b != b1) {
      const int i = bonds[2 * b], j = bonds[2 * b + 1];
      if (row2[i] != row2[j]) {
        const bool shared = i == i1 || i == j1 || j == i1 || j == j1;
        keep = shared || b > b1;
        twice = !shared;
      }
    }
    const unsigned long long m = __ballot(keep);
    const int pos = __popcll(m & ((1ull << lane) - 1ull));
    if (keep) list[n + pos] = (int16_t)(b | (twice ? kPairTwice : 0));
    n += __popcll(m);
  }
  wave_sync_lds();
  return n;
}

}  // namespace nqs
