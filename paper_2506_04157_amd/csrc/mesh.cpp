// Host-side geometry (see mesh.hpp).
#include "mesh.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <stdexcept>

namespace stk {

// Micro-tet types of the structured refinement, vertex offsets in P1 lattice
// units relative to the cube origin p: 0 = "up" p+{0,a,b,c}; 1..4 = the
// octahedron p+{a,b,c,a+b,a+c,b+c} cut along its diagonal b <-> a+c; 5 =
// "down" p+{a+b,a+c,b+c,a+b+c}.
const int TYPE_OFF[6][4][3] = {
    {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{0, 1, 0}, {1, 0, 1}, {1, 0, 0}, {1, 1, 0}},
    {{0, 1, 0}, {1, 0, 1}, {1, 1, 0}, {0, 1, 1}},
    {{0, 1, 0}, {1, 0, 1}, {0, 1, 1}, {0, 0, 1}},
    {{0, 1, 0}, {1, 0, 1}, {0, 0, 1}, {1, 0, 0}},
    {{1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}},
};
const int EDGE_V[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

MacroMesh make_cube() {
  MacroMesh mm;
  mm.kind = 0;
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y)
      for (int z = 0; z < 2; ++z) {
        mm.V.push_back(x);
        mm.V.push_back(y);
        mm.V.push_back(z);
        mm.layer.push_back(-1);
      }
  // Kuhn paths 0 -> e_s1 -> e_s1+e_s2 -> (1,1,1), permutations in lexicographic order
  const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (auto& s : perms) {
    int p[3] = {0, 0, 0};
    std::array<int, 4> t;
    t[0] = 0;
    for (int k = 0; k < 3; ++k) {
      p[s[k]] = 1;
      t[k + 1] = 4 * p[0] + 2 * p[1] + p[2];
    }
    mm.tets.push_back(t);
  }
  return mm;
}

void icosahedron(double ico[12][3], std::vector<std::array<int, 3>>& faces) {
  const double phi = (1.0 + std::sqrt(5.0)) / 2.0;
  const double raw[12][3] = {{0, 1, phi},  {0, -1, phi},  {0, 1, -phi},  {0, -1, -phi},
                             {1, phi, 0},  {-1, phi, 0},  {1, -phi, 0},  {-1, -phi, 0},
                             {phi, 0, 1},  {-phi, 0, 1},  {phi, 0, -1},  {-phi, 0, -1}};
  for (int i = 0; i < 12; ++i) {
    double n = std::sqrt(raw[i][0] * raw[i][0] + raw[i][1] * raw[i][1] + raw[i][2] * raw[i][2]);
    for (int d = 0; d < 3; ++d) ico[i][d] = raw[i][d] / n;
  }
  auto dist = [&](int i, int j) {
    double s = 0;
    for (int d = 0; d < 3; ++d) s += (ico[i][d] - ico[j][d]) * (ico[i][d] - ico[j][d]);
    return std::sqrt(s);
  };
  double emin = 10;
  for (int i = 0; i < 12; ++i)
    for (int j = i + 1; j < 12; ++j) emin = std::min(emin, dist(i, j));
  faces.clear();
  for (int i = 0; i < 12; ++i)
    for (int j = i + 1; j < 12; ++j)
      for (int k = j + 1; k < 12; ++k)
        if (std::fabs(dist(i, j) - emin) < 1e-9 && std::fabs(dist(j, k) - emin) < 1e-9 &&
            std::fabs(dist(i, k) - emin) < 1e-9)
          faces.push_back({i, j, k});
  if (faces.size() != 20) throw std::runtime_error("icosahedron faces");
}

MacroMesh make_shell(int n_tan, int n_rad, double r_in, double r_out) {
  double ico[12][3];
  std::vector<std::array<int, 3>> faces;
  icosahedron(ico, faces);

  // sphere points keyed by their integer weights over the 12 icosahedron vertices
  using Key = std::array<int, 12>;
  std::map<Key, int> keymap;
  std::vector<Key> keys;
  std::vector<std::array<int, 3>> tris;   // by key index (pre-sort)
  for (auto& f : faces) {
    std::map<std::pair<int, int>, int> idx;
    for (int i = 0; i <= n_tan; ++i)
      for (int j = 0; j <= n_tan - i; ++j) {
        Key w{};
        w[f[0]] += i;
        w[f[1]] += j;
        w[f[2]] += n_tan - i - j;
        auto it = keymap.find(w);
        int id;
        if (it == keymap.end()) {
          id = (int)keys.size();
          keymap[w] = id;
          keys.push_back(w);
        } else {
          id = it->second;
        }
        idx[{i, j}] = id;
      }
    for (int i = 0; i < n_tan; ++i)
      for (int j = 0; j < n_tan - i; ++j) {
        tris.push_back({idx[{i, j}], idx[{i + 1, j}], idx[{i, j + 1}]});
        if (i + j <= n_tan - 2) tris.push_back({idx[{i + 1, j}], idx[{i, j + 1}], idx[{i + 1, j + 1}]});
      }
  }
  // rank of each key in lexicographic order = the point id
  std::vector<int> rank(keys.size());
  {
    int r = 0;
    for (auto& kv : keymap) rank[kv.second] = r++;
  }
  const int ns = (int)keys.size();
  std::vector<double> dirs(3 * ns);
  for (int s = 0; s < ns; ++s) {
    const Key& w = keys[s];
    double v[3] = {0, 0, 0};
    for (int k = 0; k < 12; ++k)
      for (int d = 0; d < 3; ++d) v[d] += w[k] * ico[k][d];
    double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int d = 0; d < 3; ++d) dirs[3 * rank[s] + d] = v[d] / n;
  }
  MacroMesh mm;
  mm.kind = 1;
  mm.r_in = r_in;
  mm.r_out = r_out;
  mm.n_rad = n_rad;
  for (int k = 0; k <= n_rad; ++k) {
    double r = r_in + (r_out - r_in) * k / n_rad;
    for (int s = 0; s < ns; ++s) {
      for (int d = 0; d < 3; ++d) mm.V.push_back(r * dirs[3 * s + d]);
      mm.layer.push_back(k);
    }
  }
  for (auto& t : tris) {
    int s[3] = {rank[t[0]], rank[t[1]], rank[t[2]]};
    std::sort(s, s + 3);
    for (int k = 0; k < n_rad; ++k) {
      int a0 = s[0] + k * ns, a1 = s[1] + k * ns, a2 = s[2] + k * ns;
      int b0 = s[0] + (k + 1) * ns, b1 = s[1] + (k + 1) * ns, b2 = s[2] + (k + 1) * ns;
      mm.tets.push_back({a0, a1, a2, b2});
      mm.tets.push_back({a0, a1, b1, b2});
      mm.tets.push_back({a0, b0, b1, b2});
    }
  }
  return mm;
}

Topology build_topology(const MacroMesh& mm) {
  Topology t;
  const int nm = mm.nm();
  std::map<std::array<int, 3>, int> fmap;
  std::map<std::array<int, 2>, int> emap;
  std::vector<int> fcount;
  t.mface.resize(nm);
  t.medge.resize(nm);
  for (int m = 0; m < nm; ++m) {
    const auto& v = mm.tets[m];
    for (int f = 0; f < 4; ++f) {
      std::array<int, 3> k;
      int c = 0;
      for (int i = 0; i < 4; ++i)
        if (i != f) k[c++] = v[i];
      std::sort(k.begin(), k.end());
      auto it = fmap.find(k);
      if (it == fmap.end()) {
        int id = (int)t.faces.size();
        fmap[k] = id;
        t.faces.push_back(k);
        fcount.push_back(1);
        t.fowner.push_back(m);
        t.mface[m][f] = id;
      } else {
        fcount[it->second]++;
        t.mface[m][f] = it->second;
      }
    }
    for (int e = 0; e < 6; ++e) {
      std::array<int, 2> k = {v[EDGE_V[e][0]], v[EDGE_V[e][1]]};
      if (k[0] > k[1]) std::swap(k[0], k[1]);
      auto it = emap.find(k);
      if (it == emap.end()) {
        int id = (int)t.edges.size();
        emap[k] = id;
        t.edges.push_back(k);
        t.eowner.push_back(m);
        t.medge[m][e] = id;
      } else {
        t.medge[m][e] = it->second;
      }
    }
  }
  t.vowner.assign(mm.nv(), -1);
  for (int m = 0; m < nm; ++m)
    for (int i = 0; i < 4; ++i)
      if (t.vowner[mm.tets[m][i]] < 0) t.vowner[mm.tets[m][i]] = m;
  t.fkind.assign(t.faces.size(), 0);
  t.ekind.assign(t.edges.size(), 0);
  t.vkind.assign(mm.nv(), 0);
  for (size_t f = 0; f < t.faces.size(); ++f) {
    if (fcount[f] != 1) continue;
    int kind = 1;
    if (mm.kind == 1) {
      const auto& k = t.faces[f];
      int l0 = mm.layer[k[0]];
      if (l0 != mm.layer[k[1]] || l0 != mm.layer[k[2]] || (l0 != 0 && l0 != mm.n_rad))
        throw std::runtime_error("boundary face not on a sphere");
      kind = (l0 == 0) ? 1 : 2;
    }
    t.fkind[f] = kind;
    const auto& k = t.faces[f];
    for (int a = 0; a < 3; ++a) {
      t.vkind[k[a]] = kind;
      for (int b = a + 1; b < 3; ++b) t.ekind[emap[{k[a], k[b]}]] = kind;
    }
  }
  t.bkind.assign((size_t)nm * 16, 0);
  t.own.assign((size_t)nm * 16, 0);
  for (int m = 0; m < nm; ++m) {
    for (int mask = 1; mask < 16; ++mask) {
      int cnt = __builtin_popcount(mask);
      int kind = 0, owner = m;
      if (cnt == 1) {
        int v = __builtin_ctz(mask);
        kind = t.vkind[mm.tets[m][v]];
        owner = t.vowner[mm.tets[m][v]];
      } else if (cnt == 2) {
        int i = __builtin_ctz(mask), j = 31 - __builtin_clz(mask);
        int e = 0;
        for (; e < 6; ++e)
          if (EDGE_V[e][0] == i && EDGE_V[e][1] == j) break;
        kind = t.ekind[t.medge[m][e]];
        owner = t.eowner[t.medge[m][e]];
      } else if (cnt == 3) {
        int f = __builtin_ctz(~mask & 15);
        kind = t.fkind[t.mface[m][f]];
        owner = t.fowner[t.mface[m][f]];
      }
      t.bkind[(size_t)m * 16 + mask] = (uint8_t)kind;
      t.own[(size_t)m * 16 + mask] = (uint8_t)(owner == m);
    }
  }
  return t;
}

std::vector<double> macro_geometry(const MacroMesh& mm) {
  const int nm = mm.nm();
  std::vector<double> G((size_t)nm * 16, 0.0);
  for (int m = 0; m < nm; ++m) {
    double v[4][3];
    for (int i = 0; i < 4; ++i)
      for (int d = 0; d < 3; ++d) v[i][d] = mm.V[3 * mm.tets[m][i] + d];
    double* g = &G[(size_t)m * 16];
    for (int d = 0; d < 3; ++d) g[d] = v[0][d];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) g[3 + 3 * r + c] = v[c + 1][r] - v[0][r];
    if (mm.kind == 1) {
      // s(x) = gs.x + s0 interpolates the vertex radii: solve [v_i^T 1][gs; s0] = |v_i|
      double M[4][5];
      for (int i = 0; i < 4; ++i) {
        for (int d = 0; d < 3; ++d) M[i][d] = v[i][d];
        M[i][3] = 1.0;
        M[i][4] = std::sqrt(v[i][0] * v[i][0] + v[i][1] * v[i][1] + v[i][2] * v[i][2]);
      }
      for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
          if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
        for (int k = 0; k < 5; ++k) std::swap(M[c][k], M[piv][k]);
        for (int r = 0; r < 4; ++r) {
          if (r == c) continue;
          double f = M[r][c] / M[c][c];
          for (int k = c; k < 5; ++k) M[r][k] -= f * M[c][k];
        }
      }
      for (int c = 0; c < 4; ++c) g[12 + c] = M[c][4] / M[c][c];
    }
  }
  return G;
}

static void inv3(const double A[3][3], double R[3][3], double* det) {
  double d = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
             A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
             A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  R[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / d;
  R[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / d;
  R[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / d;
  R[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / d;
  R[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / d;
  R[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / d;
  R[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / d;
  R[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / d;
  R[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / d;
  *det = d;
}

Level build_level(const MacroMesh& mm, const Topology& top, int L) {
  Level lv;
  lv.L = L;
  lv.n = 1 << L;
  const int nm = mm.nm();
  const std::vector<double> geo = macro_geometry(mm);
  for (int pass = 0; pass < 2; ++pass) {
    const int m = pass == 0 ? 2 * lv.n : lv.n;   // lattice side (P2 then P1)
    const int64_t ci = (int64_t)(m - 1) * (m - 2) * (m - 3) / 6;
    const int64_t fi = (int64_t)(m - 1) * (m - 2) / 2;
    const int64_t ei = m - 1;
    const int64_t faceBase = (int64_t)nm * ci;
    const int64_t edgeBase = faceBase + (int64_t)top.faces.size() * fi;
    const int64_t vertBase = edgeBase + (int64_t)top.edges.size() * ei;
    const int64_t total = vertBase + mm.nv();
    if (total >= (int64_t)INT32_MAX) throw std::runtime_error("node count exceeds signed 32-bit indices");
    const int64_t nloc = tet_count(m);
    std::vector<uint32_t>& l2g = pass == 0 ? lv.l2g2 : lv.l2g1;
    l2g.resize((size_t)nm * nloc);
    // local lattice classification (same for every macro)
    std::vector<int> loc_w(4 * nloc), loc_int(nloc, -1);
    {
      int64_t l = 0, ni = 0;
      for (int K = 0; K <= m; ++K)
        for (int J = 0; J <= m - K; ++J)
          for (int I = 0; I <= m - J - K; ++I, ++l) {
            int w[4] = {m - I - J - K, I, J, K};
            for (int k = 0; k < 4; ++k) loc_w[4 * l + k] = w[k];
            if (w[0] > 0 && I > 0 && J > 0 && K > 0) {
              // the kernels compute a macro-interior index in closed form as
              // the lattice index of (I-1, J-1, K-1) in the side m-4 lattice
              if (lattice_loc(I - 1, J - 1, K - 1, m - 4) != ni)
                throw std::runtime_error("interior numbering is not the shifted lattice order");
              loc_int[l] = (int)ni++;
            }
          }
    }
    for (int mc = 0; mc < nm; ++mc) {
      const auto& tv = mm.tets[mc];
      for (int64_t l = 0; l < nloc; ++l) {
        const int* w = &loc_w[4 * l];
        int mask = (w[0] > 0) | ((w[1] > 0) << 1) | ((w[2] > 0) << 2) | ((w[3] > 0) << 3);
        int cnt = __builtin_popcount(mask);
        int64_t gid;
        if (cnt == 4) {
          gid = (int64_t)mc * ci + loc_int[l];
        } else if (cnt == 3) {
          int f = __builtin_ctz(~mask & 15);
          int gf = top.mface[mc][f];
          const auto& fv = top.faces[gf];
          int wv[3];
          for (int a = 0; a < 3; ++a)
            for (int k = 0; k < 4; ++k)
              if (tv[k] == fv[a]) wv[a] = w[k];
          int64_t kk = wv[2] - 1;
          gid = faceBase + (int64_t)gf * fi + kk * (m - 1) - kk * (kk + 1) / 2 + (wv[1] - 1);
        } else if (cnt == 2) {
          int i = __builtin_ctz(mask), j = 31 - __builtin_clz(mask);
          int e = 0;
          for (; e < 6; ++e)
            if (EDGE_V[e][0] == i && EDGE_V[e][1] == j) break;
          int ge = top.medge[mc][e];
          int hi = top.edges[ge][1];
          int whi = (tv[i] == hi) ? w[i] : w[j];
          gid = edgeBase + (int64_t)ge * ei + (whi - 1);
        } else {
          gid = vertBase + tv[__builtin_ctz(mask)];
        }
        l2g[(size_t)mc * nloc + l] = (uint32_t)gid;
        const int kind = top.bkind[(size_t)mc * 16 + mask];
        if (pass == 0 && kind != 0 && top.own[(size_t)mc * 16 + mask]) {
          double xt[3];
          for (int d = 0; d < 3; ++d)
            xt[d] = (w[0] * mm.V[3 * tv[0] + d] + w[1] * mm.V[3 * tv[1] + d] +
                     w[2] * mm.V[3 * tv[2] + d] + w[3] * mm.V[3 * tv[3] + d]) / m;
          double r = std::sqrt(xt[0] * xt[0] + xt[1] * xt[1] + xt[2] * xt[2]);
          lv.bnode.push_back((uint32_t)gid);
          lv.bkind.push_back((uint8_t)kind);
          for (int d = 0; d < 3; ++d) lv.bnormal.push_back(r > 0 ? xt[d] / r : 0.0);
        }
      }
    }
    if (pass == 0) {
      lv.n2 = total;
      lv.nloc2 = nloc;
    } else {
      lv.n1 = total;
      lv.nloc1 = nloc;
    }
  }
  // inverse Jacobians of the 6 micro-tet types per macro
  lv.tinv.assign((size_t)nm * 60, 0.0);
  for (int mc = 0; mc < nm; ++mc) {
    const double* g = &geo[(size_t)mc * 16];
    for (int t = 0; t < 6; ++t) {
      double JF[3][3];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double s = 0;
          for (int k = 0; k < 3; ++k) s += g[3 + 3 * r + k] * (TYPE_OFF[t][c + 1][k] - TYPE_OFF[t][0][k]);
          JF[r][c] = s / lv.n;
        }
      double R[3][3], det;
      inv3(JF, R, &det);
      double* o = &lv.tinv[((size_t)mc * 6 + t) * 10];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) o[3 * r + c] = R[r][c];
      o[9] = std::fabs(det);
    }
  }
  const int nb = (lv.n - 1) / TILE;
  for (int bk = 0; bk <= nb; ++bk)
    for (int bj = 0; bj <= nb - bk; ++bj)
      for (int bi = 0; bi <= nb - bj - bk; ++bi) {
        lv.tiles.push_back(TILE * bi);
        lv.tiles.push_back(TILE * bj);
        lv.tiles.push_back(TILE * bk);
      }
  return lv;
}

Sweep build_sweep(int n, int nstrips) {
  Sweep sw;
  const int m2 = 2 * n;
  if (nstrips > n) nstrips = n;
  if (nstrips < 1) nstrips = 1;
  // balance element counts: cube row py holds about (n - py)(n - py + 1)/2 cubes
  std::vector<double> w(n);
  double tot = 0;
  for (int j = 0; j < n; ++j) tot += (w[j] = 0.5 * (n - j) * (n - j + 1));
  std::vector<int> cuts = {0};
  double acc = 0;
  for (int j = 0; j < n && (int)cuts.size() < nstrips; ++j) {
    acc += w[j];
    if (acc >= tot * cuts.size() / nstrips && j + 1 < n) cuts.push_back(j + 1);
  }
  cuts.push_back(n);
  sw.nstrips = (int)cuts.size() - 1;
  for (int s = 0; s < sw.nstrips; ++s) {
    sw.strip.push_back(cuts[s]);
    sw.strip.push_back(cuts[s + 1]);
  }
  auto is_cut = [&](int j) {   // internal strip boundary row (P1 units)
    for (int s = 1; s < sw.nstrips; ++s)
      if (cuts[s] == j) return true;
    return false;
  };
  int nsh2 = 0, nsh1 = 0;
  for (int st = 0; st < sw.nstrips; ++st) {
    const int j0 = cuts[st], j1 = cuts[st + 1];
    for (int K = 0; K <= m2; ++K) {
      sw.poff2.push_back((int)sw.plist2.size() / 2);
      int cnt = 0;
      for (int J = 2 * j0; J <= std::min(2 * j1, m2 - K); ++J)
        for (int I = 0; I <= m2 - K - J; ++I) {
          const bool bnd = (m2 - I - J - K) == 0 || I == 0 || J == 0 || K == 0;
          const bool shared = bnd || ((J % 2) == 0 && is_cut(J / 2));
          sw.plist2.push_back(I | (J << 10) | (K << 20));
          sw.plist2.push_back(shared ? nsh2++ : -1);
          ++cnt;
        }
      sw.cap2 = std::max(sw.cap2, cnt);
    }
    sw.poff2.push_back((int)sw.plist2.size() / 2);
    for (int k = 0; k <= n; ++k) {
      sw.poff1.push_back((int)sw.plist1.size() / 2);
      int cnt = 0;
      for (int J = j0; J <= std::min(j1, n - k); ++J)
        for (int I = 0; I <= n - k - J; ++I) {
          const bool bnd = (n - I - J - k) == 0 || I == 0 || J == 0 || k == 0;
          const bool shared = bnd || is_cut(J);
          sw.plist1.push_back(I | (J << 10) | (k << 20));
          sw.plist1.push_back(shared ? nsh1++ : -1);
          ++cnt;
        }
      sw.cap1 = std::max(sw.cap1, cnt);
    }
    sw.poff1.push_back((int)sw.plist1.size() / 2);
    for (int k = 0; k < n; ++k) {
      sw.eoff.push_back((int)sw.elist.size());
      for (int t = 0; t < 6; ++t) {
        const int lim = t == 0 ? n - 1 : (t == 5 ? n - 3 : n - 2);
        for (int py = j0; py < j1; ++py)
          for (int px = 0; px + py + k <= lim; ++px) sw.elist.push_back(t | (px << 3) | (py << 13));
      }
    }
    sw.eoff.push_back((int)sw.elist.size());
  }
  sw.nsh2 = nsh2;
  sw.nsh1 = nsh1;
  // LDS ring positions of every element's nodes: position of (I, J) within the
  // strip part (rows J >= a) of plane K of a lattice of side m, plus the slot
  if (3 * sw.cap2 > 65535 || 2 * sw.cap1 > 65535) throw std::runtime_error("sweep ring exceeds 16-bit positions");
  auto ppos = [](int K, int J, int I, int m, int a) {
    const int s = m - K;
    return (J - a) * (s + 1) - (J * (J - 1) - a * (a - 1)) / 2 + I;
  };
  sw.etab.reserve(sw.elist.size() * 8);
  for (int st = 0; st < sw.nstrips; ++st) {
    const int j0 = cuts[st];
    for (int k = 0; k < n; ++k)
      for (int e = sw.eoff[st * (n + 1) + k]; e < sw.eoff[st * (n + 1) + k + 1]; ++e) {
        const int pk = sw.elist[e];
        const int t = pk & 7, px = (pk >> 3) & 1023, py = pk >> 13;
        int p2[10], p1[4];
        for (int v = 0; v < 4; ++v) {
          const int I = px + TYPE_OFF[t][v][0], J = py + TYPE_OFF[t][v][1], K = k + TYPE_OFF[t][v][2];
          p1[v] = (K % 2) * sw.cap1 + ppos(K, J, I, n, j0);
          p2[v] = ((2 * K) % 3) * sw.cap2 + ppos(2 * K, 2 * J, 2 * I, m2, 2 * j0);
        }
        for (int ed = 0; ed < 6; ++ed) {
          const int a = EDGE_V[ed][0], b = EDGE_V[ed][1];
          const int I = 2 * px + TYPE_OFF[t][a][0] + TYPE_OFF[t][b][0];
          const int J = 2 * py + TYPE_OFF[t][a][1] + TYPE_OFF[t][b][1];
          const int K = 2 * k + TYPE_OFF[t][a][2] + TYPE_OFF[t][b][2];
          p2[4 + ed] = (K % 3) * sw.cap2 + ppos(K, J, I, m2, 2 * j0);
        }
        for (int w = 0; w < 5; ++w) sw.etab.push_back(p2[2 * w] | (p2[2 * w + 1] << 16));
        sw.etab.push_back(p1[0] | (p1[1] << 16));
        sw.etab.push_back(p1[2] | (p1[3] << 16));
        sw.etab.push_back(t);
      }
  }
  return sw;
}

void build_gather(const MacroMesh& mm, const Level& lv, const Sweep& sw, int which, std::vector<uint32_t>& node,
                  std::vector<int>& ptr, std::vector<int>& slot) {
  const int nm = mm.nm();
  const int m = which == 2 ? 2 * lv.n : lv.n;
  const int64_t nloc = which == 2 ? lv.nloc2 : lv.nloc1;
  const std::vector<uint32_t>& l2g = which == 2 ? lv.l2g2 : lv.l2g1;
  const std::vector<int>& pl = which == 2 ? sw.plist2 : sw.plist1;
  const int nsh = which == 2 ? sw.nsh2 : sw.nsh1;
  const int64_t ntot = which == 2 ? lv.n2 : lv.n1;
  // local (entry -> loc) for the shared entries
  std::vector<std::pair<int, int>> sh;   // (loc, slot)
  for (size_t e = 0; e < pl.size() / 2; ++e) {
    if (pl[2 * e + 1] < 0) continue;
    const int pk = pl[2 * e];
    const int I = pk & 1023, J = (pk >> 10) & 1023, K = pk >> 20;
    sh.push_back({(int)lattice_loc(I, J, K, m), pl[2 * e + 1]});
  }
  std::vector<int> cnt(ntot + 1, 0);
  for (int mc = 0; mc < nm; ++mc)
    for (auto& e : sh) cnt[l2g[(size_t)mc * nloc + e.first] + 1]++;
  // compact: only nodes with at least one slot
  node.clear();
  ptr.assign(1, 0);
  std::vector<int> pos(ntot, -1);
  for (int64_t g = 0; g < ntot; ++g)
    if (cnt[g + 1] > 0) {
      pos[g] = ptr.back();
      node.push_back((uint32_t)g);
      ptr.push_back(ptr.back() + cnt[g + 1]);
    }
  slot.assign(ptr.back(), 0);
  for (int mc = 0; mc < nm; ++mc)
    for (auto& e : sh) {
      const uint32_t g = l2g[(size_t)mc * nloc + e.first];
      slot[pos[g]++] = (int)((int64_t)mc * nsh + e.second);
    }
  // pos[g] now points past the node's range; a node's slots are in macro
  // order.  Order the nodes by their first slot, so that neighbouring threads
  // of the gather read neighbouring slots (the slots of one macro face are
  // contiguous in both of its macros).
  const size_t nn = node.size();
  std::vector<int> order(nn);
  for (size_t i = 0; i < nn; ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return slot[ptr[a]] < slot[ptr[b]]; });
  std::vector<uint32_t> node2(nn);
  std::vector<int> ptr2(1, 0), slot2;
  slot2.reserve(slot.size());
  for (size_t i = 0; i < nn; ++i) {
    const int a = order[i];
    node2[i] = node[a];
    for (int k = ptr[a]; k < ptr[a + 1]; ++k) slot2.push_back(slot[k]);
    ptr2.push_back((int)slot2.size());
  }
  node.swap(node2);
  ptr.swap(ptr2);
  slot.swap(slot2);
}

void level_coords(const MacroMesh& mm, const Topology& top, const Level& lv, int which, double* X,
                  uint8_t* flags) {
  const int nm = mm.nm();
  const int m = which == 2 ? 2 * lv.n : lv.n;
  const int64_t nloc = which == 2 ? lv.nloc2 : lv.nloc1;
  const std::vector<uint32_t>& l2g = which == 2 ? lv.l2g2 : lv.l2g1;
  const std::vector<double> geo = macro_geometry(mm);
  for (int mc = 0; mc < nm; ++mc) {
    const auto& tv = mm.tets[mc];
    const double* g = &geo[(size_t)mc * 16];
    int64_t l = 0;
    for (int K = 0; K <= m; ++K)
      for (int J = 0; J <= m - K; ++J)
        for (int I = 0; I <= m - J - K; ++I, ++l) {
          const int w[4] = {m - I - J - K, I, J, K};
          const int mask = (w[0] > 0) | ((w[1] > 0) << 1) | ((w[2] > 0) << 2) | ((w[3] > 0) << 3);
          if (!top.own[(size_t)mc * 16 + mask]) continue;
          const uint32_t gid = l2g[(size_t)mc * nloc + l];
          if (flags) flags[gid] = top.bkind[(size_t)mc * 16 + mask];
          if (!X) continue;
          double xt[3];
          for (int d = 0; d < 3; ++d)
            xt[d] = (w[0] * mm.V[3 * tv[0] + d] + w[1] * mm.V[3 * tv[1] + d] + w[2] * mm.V[3 * tv[2] + d] +
                     w[3] * mm.V[3 * tv[3] + d]) / m;
          double f = 1.0;
          if (mm.kind == 1) {
            double s = g[12] * xt[0] + g[13] * xt[1] + g[14] * xt[2] + g[15];
            f = s / std::sqrt(xt[0] * xt[0] + xt[1] * xt[1] + xt[2] * xt[2]);
          }
          for (int d = 0; d < 3; ++d) X[3 * (size_t)gid + d] = xt[d] * f;
        }
  }
}

}  // namespace stk

namespace stk {

P1Stencil build_p1_stencil(int n) {
  P1Stencil st;
  // directions: the node itself, then every vertex difference that occurs in a micro-tet type
  std::vector<std::array<int, 3>> dirs = {{0, 0, 0}};
  auto dir_of = [&](int a, int b, int c) {
    for (size_t d = 0; d < dirs.size(); ++d)
      if (dirs[d][0] == a && dirs[d][1] == b && dirs[d][2] == c) return (int)d;
    return -1;
  };
  for (int t = 0; t < 6; ++t)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        if (i == j) continue;
        const int a = TYPE_OFF[t][j][0] - TYPE_OFF[t][i][0], b = TYPE_OFF[t][j][1] - TYPE_OFF[t][i][1],
                  c = TYPE_OFF[t][j][2] - TYPE_OFF[t][i][2];
        if (dir_of(a, b, c) < 0) dirs.push_back({a, b, c});
      }
  if ((int)dirs.size() != NDIR1) throw std::runtime_error("unexpected lattice edge directions");
  // order: the node itself, the 7 directions that are lexicographically
  // positive, then their negatives in the same order (direction d + 7 = -d)
  {
    std::vector<std::array<int, 3>> pos;
    for (size_t d = 1; d < dirs.size(); ++d)
      if (dirs[d] > std::array<int, 3>{0, 0, 0}) pos.push_back(dirs[d]);
    std::sort(pos.begin(), pos.end());
    if (pos.size() != 7) throw std::runtime_error("lattice edge directions are not symmetric");
    dirs.assign(1, {0, 0, 0});
    for (auto& d : pos) dirs.push_back(d);
    for (auto& d : pos) dirs.push_back({-d[0], -d[1], -d[2]});
  }
  for (int d = 0; d < NDIR1; ++d)
    for (int k = 0; k < 3; ++k) st.dir[d][k] = dirs[d][k];
  const int64_t nloc = (int64_t)(n + 1) * (n + 2) * (n + 3) / 6;
  st.nb.assign((size_t)NDIR1 * nloc, 0);
  for (int K = 0; K <= n; ++K)
    for (int J = 0; J + K <= n; ++J)
      for (int I = 0; I + J + K <= n; ++I) {
        const int64_t t = lattice_loc(I, J, K, n);
        for (int d = 0; d < NDIR1; ++d) {
          const int a = I + dirs[d][0], b = J + dirs[d][1], c = K + dirs[d][2];
          const bool in = a >= 0 && b >= 0 && c >= 0 && a + b + c <= n;
          st.nb[(size_t)d * nloc + t] = (int16_t)(in ? lattice_loc(a, b, c, n) : nloc);
        }
      }
  // slots: those of a one-strip sweep (exactly the macro-boundary nodes)
  st.slots = build_sweep(n, 1);
  st.nsh = st.slots.nsh1;
  st.dst.assign(nloc, -1);
  for (size_t e = 0; e < st.slots.plist1.size() / 2; ++e) {
    const int pk = st.slots.plist1[2 * e];
    st.dst[lattice_loc(pk & 1023, (pk >> 10) & 1023, pk >> 20, n)] = st.slots.plist1[2 * e + 1];
  }
  // micro-tets containing each node, in a fixed order
  std::vector<std::vector<std::pair<int, int>>> inc(nloc);
  for (int t = 0; t < 6; ++t) {
    const int lim = t == 0 ? n - 1 : (t == 5 ? n - 3 : n - 2);
    for (int pz = 0; pz < n; ++pz)
      for (int py = 0; py < n; ++py)
        for (int px = 0; px + py + pz <= lim; ++px) {
          const int pk = t | (px << 3) | (py << 13) | (pz << 23);
          for (int v = 0; v < 4; ++v) {
            int code = v;
            for (int w = 0; w < 4; ++w) {
              const int d = dir_of(TYPE_OFF[t][w][0] - TYPE_OFF[t][v][0], TYPE_OFF[t][w][1] - TYPE_OFF[t][v][1],
                                   TYPE_OFF[t][w][2] - TYPE_OFF[t][v][2]);
              code |= d << (2 + 4 * w);
            }
            inc[lattice_loc(px + TYPE_OFF[t][v][0], py + TYPE_OFF[t][v][1], pz + TYPE_OFF[t][v][2], n)].push_back(
                {pk, code});
          }
        }
  }
  st.inc_ptr.assign(1, 0);
  for (int64_t t = 0; t < nloc; ++t) {
    for (auto& e : inc[t]) {
      st.inc.push_back(e.first);
      st.inc.push_back(e.second);
    }
    st.inc_ptr.push_back((int)(st.inc.size() / 2));
  }
  return st;
}

}  // namespace stk

namespace stk {

TransferTable build_transfer_table(const Level& coarse) {
  TransferTable tt;
  const int nc = coarse.n, mf2 = 4 * nc;
  constexpr int B2h = 2 * TILE + 1, BFh = 4 * TILE + 1;
  // inverse of the (unimodular) vertex-difference matrix of each type
  int tinv[6][3][3];
  for (int t = 0; t < 6; ++t) {
    double M[3][3], Mi[3][3], det;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) M[r][c] = TYPE_OFF[t][c + 1][r] - TYPE_OFF[t][0][r];
    inv3(M, Mi, &det);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) tinv[t][r][c] = (int)std::lround(Mi[r][c]);
  }
  const int ntiles = (int)coarse.tiles.size() / 3;
  // Entry order within a tile: fine points inside the macro first (a
  // wavefront of them loads no index table), then those on its boundary;
  // lattice order within each group (rows of consecutive fine nodes)
  std::vector<std::pair<int64_t, std::array<int, 8>>> ent;
  for (int ti = 0; ti < ntiles; ++ti) {
    tt.off.push_back((int)(tt.tab.size() / 8));
    ent.clear();
    const int ox = coarse.tiles[3 * ti], oy = coarse.tiles[3 * ti + 1], oz = coarse.tiles[3 * ti + 2];
    const int lox = ox > 0, loy = oy > 0, loz = oz > 0;
    for (int az = loz; az < BFh; ++az)
      for (int ay = loy; ay < BFh; ++ay)
        for (int ax = lox; ax < BFh; ++ax) {
          const int JX = 4 * ox + ax, JY = 4 * oy + ay, JZ = 4 * oz + az;
          if (JX + JY + JZ > mf2) continue;
          // coarse cube and quarter position inside it
          const int px = JX > 0 ? (JX - 1) >> 2 : 0, py = JY > 0 ? (JY - 1) >> 2 : 0, pz = JZ > 0 ? (JZ - 1) >> 2 : 0;
          const int fx = JX - 4 * px, fy = JY - 4 * py, fz = JZ - 4 * pz;
          const int sum = fx + fy + fz;
          const int t0 = sum <= 4 ? 0 : (sum <= 8 ? 1 : 5), t1 = sum <= 4 ? 0 : (sum <= 8 ? 4 : 5);
          int type = -1, q[4] = {0, 0, 0, 0};
          for (int t = t0; t <= t1 && type < 0; ++t) {
            const int rx = fx - 4 * TYPE_OFF[t][0][0], ry = fy - 4 * TYPE_OFF[t][0][1], rz = fz - 4 * TYPE_OFF[t][0][2];
            int l[4];
            for (int r = 0; r < 3; ++r) l[r + 1] = tinv[t][r][0] * rx + tinv[t][r][1] * ry + tinv[t][r][2] * rz;
            l[0] = 4 - l[1] - l[2] - l[3];
            if (l[0] >= 0 && l[1] >= 0 && l[2] >= 0 && l[3] >= 0) {
              type = t;
              for (int r = 0; r < 4; ++r) q[r] = l[r];
            }
          }
          if (type < 0) throw std::runtime_error("transfer table: point outside every coarse micro-tet");
          // P2 basis values times 8, and the brick-local indices of the coarse nodes
          int w[10], idx[10];
          for (int i = 0; i < 4; ++i) w[i] = q[i] * (q[i] - 2);
          for (int e = 0; e < 6; ++e) w[4 + e] = 2 * q[EDGE_V[e][0]] * q[EDGE_V[e][1]];
          const int cx = px - ox, cy = py - oy, cz = pz - oz;
          for (int v = 0; v < 4; ++v) {
            const int a = 2 * (cx + TYPE_OFF[type][v][0]), b = 2 * (cy + TYPE_OFF[type][v][1]),
                      c = 2 * (cz + TYPE_OFF[type][v][2]);
            idx[v] = a + B2h * (b + B2h * c);
          }
          for (int e = 0; e < 6; ++e) {
            const int i = EDGE_V[e][0], j = EDGE_V[e][1];
            const int a = 2 * cx + TYPE_OFF[type][i][0] + TYPE_OFF[type][j][0];
            const int b = 2 * cy + TYPE_OFF[type][i][1] + TYPE_OFF[type][j][1];
            const int c = 2 * cz + TYPE_OFF[type][i][2] + TYPE_OFF[type][j][2];
            idx[4 + e] = a + B2h * (b + B2h * c);
          }
          int packed[10], nnz = 0;
          for (int a = 0; a < 10; ++a)
            if (w[a] != 0) {
              if (idx[a] < 0 || idx[a] >= B2h * B2h * B2h) throw std::runtime_error("transfer table: index");
              packed[nnz++] = idx[a] | ((w[a] + 1) << 10);
            }
          for (int a = nnz; a < 10; ++a) packed[a] = 0;
          const bool interior = JX > 0 && JY > 0 && JZ > 0 && JX + JY + JZ < mf2;
          std::array<int, 8> e;
          e[0] = JX | (JY << 10) | (JZ << 20);
          e[1] = nnz;
          for (int k = 0; k < 5; ++k) e[2 + k] = packed[2 * k] | (packed[2 * k + 1] << 16);
          e[7] = 0;
          ent.emplace_back(interior ? 0 : 1, e);
        }
    std::stable_sort(ent.begin(), ent.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    for (const auto& e : ent) tt.tab.insert(tt.tab.end(), e.second.begin(), e.second.end());
  }
  tt.off.push_back((int)(tt.tab.size() / 8));
  return tt;
}

}  // namespace stk
