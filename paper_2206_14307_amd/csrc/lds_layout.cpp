// Host placement of the fused E_loc kernel's bond rows in LDS.
//
// On gfx950 a ds_read_b128 serves 16 lanes per cycle from 64 four-byte banks,
// so a wave's read takes the minimum 4 cycles only when the 16 lanes of each
// q row hit distinct 16-byte bank groups, i.e. read addresses that differ
// modulo 256 bytes.  The 16 lanes of a q row are the 16 images of a column
// block, and for the sample's bond b they read the table rows of b's images
// under the block's 16 group elements at one common column offset.  Hence the
// placement: colour every table row with one of 16 bank groups so that each
// such set of rows has distinct colours, then pack the rows so that a row of
// colour c starts at an address = c (mod 16 units of 16 bytes).
#include <algorithm>
#include <array>
#include <cstdint>
#include <vector>

#include "nqs_internal.h"

namespace nqs {

namespace {

constexpr int kGroups = 16;

struct XorShift {
  uint64_t s;
  uint64_t next() {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return s;
  }
};

// Min-conflicts local search; returns the colouring with the fewest repeated
// colours inside the sets (0 when every set is conflict-free).
std::vector<int> colour_rows(int NB, const std::vector<std::vector<int>>& sets) {
  std::vector<std::vector<int>> inc(NB);
  for (size_t s = 0; s < sets.size(); ++s)
    for (int x : sets[s]) inc[x].push_back((int)s);
  std::vector<std::array<int, kGroups>> cnt(sets.size());
  for (auto& a : cnt) a.fill(0);
  std::vector<int> col(NB, 0), used(kGroups, 0);
  // greedy start: fewest clashes, then the least used colour
  for (int x = 0; x < NB; ++x) {
    int best = 0, bestd = 1 << 30;
    for (int c = 0; c < kGroups; ++c) {
      int d = 0;
      for (int s : inc[x]) d += cnt[s][c];
      d = d * NB + used[c];
      if (d < bestd) {
        bestd = d;
        best = c;
      }
    }
    col[x] = best;
    ++used[best];
    for (int s : inc[x]) ++cnt[s][best];
  }
  auto clashes = [&](int x, int c) {
    int d = 0;
    for (int s : inc[x]) d += cnt[s][c] - (c == col[x] ? 1 : 0);
    return d;
  };
  long cost = 0;
  for (auto& a : cnt)
    for (int v : a) cost += std::max(0, v - 1);
  std::vector<int> best_col = col;
  long best_cost = cost;
  XorShift rng{0x9E3779B97F4A7C15ull};
  for (int it = 0; it < 400000 && cost > 0; ++it) {
    const int x = (int)(rng.next() % (uint64_t)NB);
    const int cur = clashes(x, col[x]);
    if (cur == 0) continue;
    int pick = col[x], pd = cur, ties = 0;
    for (int c = 0; c < kGroups; ++c) {
      if (c == col[x]) continue;
      const int d = clashes(x, c);
      if (d < pd) {
        pd = d;
        pick = c;
        ties = 1;
      } else if (d == pd && pd <= cur && rng.next() % (uint64_t)(++ties) == 0) {
        pick = c;
      }
    }
    if (pick == col[x] || pd > cur) continue;
    for (int s : inc[x]) {
      --cnt[s][col[x]];
      ++cnt[s][pick];
    }
    col[x] = pick;
    cost += pd - cur;
    if (cost < best_cost) {
      best_cost = cost;
      best_col = col;
    }
  }
  return best_col;
}

}  // namespace

std::vector<int> place_fused_rows(const Geometry& geo, int row16, int cap16) {
  const int NB = geo.NB, G = geo.G;
  std::vector<std::vector<int>> sets;
  for (int blk = 0; blk + 16 <= G; blk += 16)
    for (int b = 0; b < NB; ++b) {
      std::vector<int> s;
      for (int c = 0; c < 16; ++c) s.push_back(geo.bmap[(size_t)(blk + c) * NB + b] >> 1);
      std::sort(s.begin(), s.end());
      s.erase(std::unique(s.begin(), s.end()), s.end());
      if (s.size() > 1) sets.push_back(std::move(s));
    }
  std::sort(sets.begin(), sets.end());
  sets.erase(std::unique(sets.begin(), sets.end()), sets.end());
  const std::vector<int> col = colour_rows(NB, sets);
  std::vector<std::vector<int>> cls(kGroups);
  for (int x = NB - 1; x >= 0; --x) cls[col[x]].push_back(x);
  std::vector<int> addr(NB, -1);
  int p = 0, placed = 0;
  while (placed < NB) {
    std::vector<int>& q = cls[p % kGroups];
    if (q.empty()) {
      ++p;
      continue;
    }
    if (p + row16 > cap16) return {};
    addr[q.back()] = p;
    q.pop_back();
    p += row16;
    ++placed;
  }
  return addr;
}

}  // namespace nqs
