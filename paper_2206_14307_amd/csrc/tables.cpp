// Host construction of the lattice, bond and space-group tables (Sec. 3.1).
//
// Point operations act on the offset from site 0 (rotation centre; reading
// of the passage, whose point-group table is not in the text):
//   p0 (x,y)  p1 C4 (-y,x)  p2 C2 (-x,-y)  p3 C4^3 (y,-x)
//   p4,p5 axial mirrors (-x,y),(x,-y)   p6,p7 diagonal mirrors (y,x),(-y,-x)
// g = (t, p) has index (t_y*L + t_x)*8 + p and perm_g(i) = site(p.r_i + t).
// Characters: chi(g) = exp(-i K.t) chi_I(p), with the textbook C4v table over
// the classes (E, 2C4, C2, 2sigma_v, 2sigma_d).
#include <map>
#include <utility>

#include "nqs_internal.h"

namespace nqs {

namespace {
const int kPointMat[8][4] = {
    {1, 0, 0, 1}, {0, -1, 1, 0}, {-1, 0, 0, -1}, {0, 1, -1, 0},
    {-1, 0, 0, 1}, {1, 0, 0, -1}, {0, 1, 1, 0}, {0, -1, -1, 0}};
const int kPointClass[8] = {0, 1, 2, 1, 3, 3, 4, 4};
const int kIrrepChar[4][5] = {
    {1, 1, 1, 1, 1},     // A1
    {1, 1, 1, -1, -1},   // A2
    {1, -1, 1, 1, -1},   // B1
    {1, -1, 1, -1, 1}};  // B2
inline int wrap(int v, int L) { return ((v % L) + L) % L; }
}  // namespace

bool build_geometry(int L, double J1, double J2, int kx, int ky, int irrep, Geometry& geo,
                    std::string& err) {
  if (L < 4 || L > 10 || (L & 1)) {
    err = "L must be 4, 6, 8 or 10";
    return false;
  }
  if (irrep < 0 || irrep > 3) {
    err = "irrep must be 0 (A1), 1 (A2), 2 (B1) or 3 (B2)";
    return false;
  }
  kx = wrap(kx, L);
  ky = wrap(ky, L);
  const bool k0 = (kx == 0 && ky == 0), kpi = (kx == L / 2 && ky == L / 2);
  if (!k0 && !kpi) {
    err = "K must be (0,0) or (pi,pi): only those are invariant under C4v";
    return false;
  }
  const int N = L * L, G = 8 * N, NB = 4 * N;
  geo.L = L;
  geo.N = N;
  geo.G = G;
  geo.NB = NB;

  // bonds
  const int shift[4][2] = {{1, 0}, {0, 1}, {1, 1}, {1, -1}};
  geo.bond_i.resize(NB);
  geo.bond_j.resize(NB);
  geo.bond_J.resize(NB);
  std::map<std::pair<int, int>, int> bond_of;
  for (int kind = 0; kind < 4; ++kind)
    for (int i = 0; i < N; ++i) {
      const int x = i % L, y = i / L;
      const int j = wrap(x + shift[kind][0], L) + L * wrap(y + shift[kind][1], L);
      const int b = kind * N + i;
      geo.bond_i[b] = i;
      geo.bond_j[b] = j;
      geo.bond_J[b] = kind < 2 ? J1 : J2;
      bond_of[{std::min(i, j), std::max(i, j)}] = b;
    }
  if ((int)bond_of.size() != NB) {
    err = "internal: duplicate bonds";
    return false;
  }

  // space group
  geo.perm.resize((size_t)G * N);
  std::vector<int> inv((size_t)G * N);
  geo.chi.resize(G);
  for (int ty = 0; ty < L; ++ty)
    for (int tx = 0; tx < L; ++tx)
      for (int p = 0; p < 8; ++p) {
        const int g = (ty * L + tx) * 8 + p;
        const int* m = kPointMat[p];
        for (int i = 0; i < N; ++i) {
          const int x = i % L, y = i / L;
          const int xp = m[0] * x + m[1] * y + tx, yp = m[2] * x + m[3] * y + ty;
          const int s = wrap(xp, L) + L * wrap(yp, L);
          geo.perm[(size_t)g * N + i] = (uint8_t)s;
          inv[(size_t)g * N + s] = i;
        }
        const int sgn_t = kpi ? (((tx + ty) & 1) ? -1 : 1) : 1;
        geo.chi[g] = (double)(sgn_t * kIrrepChar[irrep][kPointClass[p]]);
      }

  // pre-image of each bond under each group element
  geo.bmap.resize((size_t)G * NB);
  for (int g = 0; g < G; ++g)
    for (int b = 0; b < NB; ++b) {
      const int l1 = inv[(size_t)g * N + geo.bond_i[b]];
      const int l2 = inv[(size_t)g * N + geo.bond_j[b]];
      auto it = bond_of.find({std::min(l1, l2), std::max(l1, l2)});
      if (it == bond_of.end()) {
        err = "internal: a group element does not map bonds to bonds";
        return false;
      }
      const int beta = it->second;
      const int flip = geo.bond_i[beta] == l1 ? 0 : 1;
      if ((beta < 2 * N) != (b < 2 * N)) {
        err = "internal: a group element mixes J1 and J2 bonds";
        return false;
      }
      geo.bmap[(size_t)g * NB + b] = 2 * beta + flip;
    }
  return true;
}

}  // namespace nqs
