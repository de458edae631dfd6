// Host-side mesh hierarchy and index structures (see mesh.hpp).
#include "mesh.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <stdexcept>

namespace cgp {

namespace {

inline int64_t edge_key(int64_t a, int64_t b, int64_t n) {
  return a < b ? a * n + b : b * n + a;
}

struct Bary {  // integer barycentric coordinates of the 3 vertices of a triangle
  uint8_t v[3][3];
};

}  // namespace

std::string validate(const Mesh& m) {
  char buf[256];
  const int64_t n = m.n_nodes, T = m.n_tris;
  if (n < 3 || T < 1) return "mesh needs at least 3 nodes and 1 triangle";
  if ((int64_t)m.xy.size() != 2 * n || (int64_t)m.tri.size() != 3 * T ||
      m.bedge.size() != 2 * m.btag.size())
    return "mesh array sizes inconsistent";
  std::vector<uint8_t> used(n, 0);
  for (int64_t t = 0; t < T; ++t) {
    const int32_t a = m.tri[3 * t], b = m.tri[3 * t + 1], c = m.tri[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= n || b >= n || c >= n) {
      snprintf(buf, sizeof buf, "triangle %lld has a vertex index out of range", (long long)t);
      return buf;
    }
    if (a == b || b == c || a == c) {
      snprintf(buf, sizeof buf, "triangle %lld repeats a vertex", (long long)t);
      return buf;
    }
    const double x0 = m.xy[2 * a], y0 = m.xy[2 * a + 1];
    const double det = (m.xy[2 * b] - x0) * (m.xy[2 * c + 1] - y0) -
                       (m.xy[2 * c] - x0) * (m.xy[2 * b + 1] - y0);
    if (!(det > 0.0) || !std::isfinite(det)) {
      snprintf(buf, sizeof buf, "triangle %lld is clockwise or degenerate", (long long)t);
      return buf;
    }
    used[a] = used[b] = used[c] = 1;
  }
  for (int64_t i = 0; i < n; ++i)
    if (!used[i]) {
      snprintf(buf, sizeof buf, "node %lld belongs to no triangle", (long long)i);
      return buf;
    }
  // directed edges: each may appear once; an undirected edge at most twice
  std::vector<int64_t> dk(3 * T);
  for (int64_t t = 0; t < T; ++t)
    for (int e = 0; e < 3; ++e) {
      const int64_t a = m.tri[3 * t + e], b = m.tri[3 * t + (e + 1) % 3];
      dk[3 * t + e] = a * n + b;
    }
  std::sort(dk.begin(), dk.end());
  if (std::adjacent_find(dk.begin(), dk.end()) != dk.end())
    return "non-conforming mesh: an edge is shared by two triangles of the same orientation";
  // boundary edges: directed edges whose reverse is absent
  std::vector<int64_t> bnd;
  for (int64_t k : dk) {
    const int64_t a = k / n, b = k % n;
    if (!std::binary_search(dk.begin(), dk.end(), b * n + a)) bnd.push_back(edge_key(a, b, n));
  }
  std::sort(bnd.begin(), bnd.end());
  std::vector<int64_t> given(m.btag.size());
  for (size_t e = 0; e < m.btag.size(); ++e) {
    const int64_t a = m.bedge[2 * e], b = m.bedge[2 * e + 1];
    if (a < 0 || b < 0 || a >= n || b >= n || a == b) return "boundary edge index out of range";
    if (m.btag[e] != 1 && m.btag[e] != 2) return "boundary tag must be 1 (Dirichlet) or 2 (natural)";
    given[e] = edge_key(a, b, n);
  }
  std::sort(given.begin(), given.end());
  if (std::adjacent_find(given.begin(), given.end()) != given.end())
    return "a boundary edge is listed twice";
  if (given != bnd) return "boundary edge list does not match the mesh boundary";
  return "";
}

Mesh refine(const Mesh& m) {
  const int64_t n = m.n_nodes, T = m.n_tris, F = 3 * T;
  std::vector<std::pair<int64_t, int32_t>> kv(F);
  for (int64_t t = 0; t < T; ++t)
    for (int e = 0; e < 3; ++e)
      kv[3 * t + e] = {edge_key(m.tri[3 * t + e], m.tri[3 * t + (e + 1) % 3], n),
                       (int32_t)(3 * t + e)};
  std::sort(kv.begin(), kv.end());
  std::vector<int32_t> gid(F);
  int32_t G = 0;
  for (int64_t i = 0; i < F; ++i) {
    if (i == 0 || kv[i].first != kv[i - 1].first) ++G;
    gid[kv[i].second] = G - 1;
  }
  // number the distinct edges in first-encounter order of (triangle, local edge)
  std::vector<int32_t> num(G, -1), ends(2 * (size_t)G);
  std::vector<int32_t> mid(F);
  int32_t next = 0;
  for (int64_t f = 0; f < F; ++f) {
    const int32_t g = gid[f];
    if (num[g] < 0) {
      num[g] = next;
      const int64_t t = f / 3, e = f % 3;
      ends[2 * next] = m.tri[3 * t + e];
      ends[2 * next + 1] = m.tri[3 * t + (e + 1) % 3];
      ++next;
    }
    mid[f] = (int32_t)(n + num[g]);
  }
  Mesh r;
  r.n_nodes = (int32_t)(n + G);
  r.n_tris = (int32_t)(4 * T);
  r.xy.resize(2 * (size_t)r.n_nodes);
  std::copy(m.xy.begin(), m.xy.end(), r.xy.begin());
  for (int32_t k = 0; k < G; ++k) {
    const int32_t a = ends[2 * k], b = ends[2 * k + 1];
    r.xy[2 * (n + k)] = 0.5 * (m.xy[2 * a] + m.xy[2 * b]);
    r.xy[2 * (n + k) + 1] = 0.5 * (m.xy[2 * a + 1] + m.xy[2 * b + 1]);
  }
  r.tri.resize(12 * (size_t)T);
  for (int64_t t = 0; t < T; ++t) {
    const int32_t a = m.tri[3 * t], b = m.tri[3 * t + 1], c = m.tri[3 * t + 2];
    const int32_t ab = mid[3 * t], bc = mid[3 * t + 1], ca = mid[3 * t + 2];
    const int32_t kids[12] = {a, ab, ca, ab, b, bc, ca, bc, c, ab, bc, ca};
    std::copy(kids, kids + 12, r.tri.begin() + 12 * t);
  }
  const size_t B = m.btag.size();
  r.bedge.resize(4 * B);
  r.btag.resize(2 * B);
  for (size_t e = 0; e < B; ++e) {
    const int32_t p = m.bedge[2 * e], q = m.bedge[2 * e + 1];
    const int64_t key = edge_key(p, q, n);
    auto it = std::lower_bound(kv.begin(), kv.end(), std::make_pair(key, (int32_t)-1));
    const int32_t mm = (int32_t)(n + num[gid[it->second]]);
    const int32_t kids[4] = {p, mm, mm, q};
    std::copy(kids, kids + 4, r.bedge.begin() + 4 * e);
    r.btag[2 * e] = r.btag[2 * e + 1] = m.btag[e];
  }
  return r;
}

Graph build_graph(const Mesh& m) {
  const int64_t n = m.n_nodes, T = m.n_tris;
  // directed pairs (i -> j, third k, orientation) : two per triangle vertex
  std::vector<int32_t> cnt(n + 1, 0);
  for (int64_t t = 0; t < 3 * T; ++t) cnt[m.tri[t] + 1] += 2;
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  struct Ent {
    int32_t j, k, ccw;
  };
  std::vector<Ent> ent(cnt[n]);
  std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t t = 0; t < T; ++t) {
    const int32_t v[3] = {m.tri[3 * t], m.tri[3 * t + 1], m.tri[3 * t + 2]};
    for (int e = 0; e < 3; ++e) {
      const int32_t i = v[e], j = v[(e + 1) % 3], k = v[(e + 2) % 3];
      ent[fill[i]++] = {j, k, 1};  // (i, j, k) counter-clockwise
      ent[fill[i]++] = {k, j, 0};  // (i, k, j) clockwise: slot (i, k), third j
    }
  }
  Graph g;
  g.rowptr.assign(n + 1, 0);
  g.col.reserve(cnt[n] / 2 + n + 8);
  g.side.reserve(cnt[n] + 2 * n + 16);
  for (int64_t i = 0; i < n; ++i) {
    std::sort(ent.begin() + cnt[i], ent.begin() + cnt[i + 1],
              [](const Ent& a, const Ent& b) { return a.j < b.j || (a.j == b.j && a.ccw > b.ccw); });
    g.col.push_back((int32_t)i);
    g.side.push_back(-1);
    g.side.push_back(-1);
    for (int32_t s = cnt[i]; s < cnt[i + 1];) {
      const int32_t j = ent[s].j;
      int32_t kc = -1, kw = -1;
      for (; s < cnt[i + 1] && ent[s].j == j; ++s) (ent[s].ccw ? kc : kw) = ent[s].k;
      g.col.push_back(j);
      g.side.push_back(kc);
      g.side.push_back(kw);
    }
    g.rowptr[i + 1] = (int32_t)g.col.size();
  }
  // greedy row tiles: <= kTileRows rows and <= kTileNnz nonzeros each
  g.tile.assign(1, 0);
  for (int64_t r = 0; r < n;) {
    const int64_t start = r;
    while (r < n && r - start < kTileRows && g.rowptr[r + 1] - g.rowptr[start] <= kTileNnz) ++r;
    if (r == start) throw std::runtime_error("a node has more than kTileNnz neighbours");
    g.tile.push_back((int32_t)r);
  }
  return g;
}

std::string build_hierarchy(const Mesh& coarse, int levels, Hierarchy& h) {
  if (levels < 0 || levels > 3) return "levels must be in 0..3";
  std::string err = validate(coarse);
  if (!err.empty()) return err;
  if ((int64_t)coarse.n_tris << (2 * levels) > (int64_t)INT32_MAX / 4)
    return "refined mesh too large for 32-bit indices";
  h.levels = levels;
  h.coarse = coarse;
  const int32_t nc = coarse.n_nodes;
  const int32_t den = 1 << levels;

  // barycentric coordinates (relative to the coarse ancestor) of the vertices
  // of the triangles of the current level, and per-node codes
  std::vector<Bary> bary(coarse.n_tris);
  for (auto& b : bary) {
    for (int v = 0; v < 3; ++v)
      for (int w = 0; w < 3; ++w) b.v[v][w] = (uint8_t)(v == w);
  }
  std::vector<int32_t> code_T, code_n;  // per node: ancestor, n1 | n2 << 16 (at denominator 2^levels)
  code_T.assign(nc, -1);
  code_n.assign(nc, 0);
  for (int32_t t = 0; t < coarse.n_tris; ++t)
    for (int v = 0; v < 3; ++v) {
      const int32_t i = coarse.tri[3 * t + v];
      if (code_T[i] < 0) {
        code_T[i] = t;
        code_n[i] = (v == 1 ? den : 0) | ((v == 2 ? den : 0) << 16);
      }
    }

  Mesh cur = coarse;
  for (int l = 0; l < levels; ++l) {
    Mesh nxt = refine(cur);
    const int32_t n0 = cur.n_nodes;
    const int scale = 1 << (levels - l - 1);  // from denominator 2^(l+1) to 2^levels
    code_T.resize(nxt.n_nodes, -1);
    code_n.resize(nxt.n_nodes, 0);
    std::vector<Bary> nb(4 * (size_t)cur.n_tris);
    for (int64_t t = 0; t < cur.n_tris; ++t) {
      const Bary& B = bary[t];
      const int32_t T = (int32_t)(t >> (2 * l));
      uint8_t m[3][3];  // midpoints of local edges (0,1), (1,2), (2,0)
      for (int w = 0; w < 3; ++w) {
        m[0][w] = B.v[0][w] + B.v[1][w];
        m[1][w] = B.v[1][w] + B.v[2][w];
        m[2][w] = B.v[2][w] + B.v[0][w];
      }
      for (int e = 0; e < 3; ++e) {
        // the new node on local edge e of t: children 0,1,2 hold it at known spots
        static const int kid[3] = {0, 1, 2}, pos[3] = {1, 2, 0};
        const int32_t node = nxt.tri[3 * (4 * t + kid[e]) + pos[e]];
        if (node >= n0 && code_T[node] < 0) {
          code_T[node] = T;
          code_n[node] = (m[e][1] * scale) | ((m[e][2] * scale) << 16);
        }
      }
      Bary c[4];
      for (int w = 0; w < 3; ++w) {
        const uint8_t A = 2 * B.v[0][w], Bv = 2 * B.v[1][w], C = 2 * B.v[2][w];
        c[0].v[0][w] = A;       c[0].v[1][w] = m[0][w]; c[0].v[2][w] = m[2][w];
        c[1].v[0][w] = m[0][w]; c[1].v[1][w] = Bv;      c[1].v[2][w] = m[1][w];
        c[2].v[0][w] = m[2][w]; c[2].v[1][w] = m[1][w]; c[2].v[2][w] = C;
        c[3].v[0][w] = m[0][w]; c[3].v[1][w] = m[1][w]; c[3].v[2][w] = m[2][w];
      }
      for (int q = 0; q < 4; ++q) nb[4 * t + q] = c[q];
    }
    bary.swap(nb);
    cur = std::move(nxt);
  }
  if (levels > 0) {
    // canonical fine numbering: the coarse nodes keep 0..N_c-1, the new nodes
    // follow stably sorted by the coarse triangle that created them
    // (code_T), so that the nodes of one coarse triangle are contiguous and
    // neighbour gathers stay local in memory
    const int32_t n = cur.n_nodes;
    std::vector<int32_t> order(n - nc);
    std::iota(order.begin(), order.end(), nc);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return code_T[a] < code_T[b]; });
    std::vector<int32_t> canon(n);
    for (int32_t i = 0; i < nc; ++i) canon[i] = i;
    for (int32_t k = 0; k < n - nc; ++k) canon[order[k]] = nc + k;
    Mesh f;
    f.n_nodes = n;
    f.n_tris = cur.n_tris;
    f.xy.resize(cur.xy.size());
    std::vector<int32_t> cT(n), cN(n);
    for (int32_t i = 0; i < n; ++i) {
      f.xy[2 * (size_t)canon[i]] = cur.xy[2 * (size_t)i];
      f.xy[2 * (size_t)canon[i] + 1] = cur.xy[2 * (size_t)i + 1];
      cT[canon[i]] = code_T[i];
      cN[canon[i]] = code_n[i];
    }
    f.tri.resize(cur.tri.size());
    for (size_t k = 0; k < cur.tri.size(); ++k) f.tri[k] = canon[cur.tri[k]];
    f.bedge.resize(cur.bedge.size());
    for (size_t k = 0; k < cur.bedge.size(); ++k) f.bedge[k] = canon[cur.bedge[k]];
    f.btag = cur.btag;
    cur = std::move(f);
    code_T.swap(cT);
    code_n.swap(cN);
  }
  h.fine = std::move(cur);
  const int32_t nf = h.fine.n_nodes;
  for (int32_t i = 0; i < nf; ++i)
    if (code_T[i] < 0) return "internal error: fine node without prolongation code";
  h.pcode.resize(2 * (size_t)nf);
  for (int32_t i = 0; i < nf; ++i) {
    h.pcode[2 * i] = code_T[i];
    h.pcode[2 * i + 1] = code_n[i];
  }
  h.gc = build_graph(h.coarse);
  h.gf = levels == 0 ? h.gc : build_graph(h.fine);

  // coarse node -> incident coarse triangles
  h.cn_ptr.assign(nc + 1, 0);
  for (int64_t k = 0; k < 3 * (int64_t)coarse.n_tris; ++k) h.cn_ptr[coarse.tri[k] + 1]++;
  for (int32_t i = 0; i < nc; ++i) h.cn_ptr[i + 1] += h.cn_ptr[i];
  h.cn_tri.resize(h.cn_ptr[nc]);
  std::vector<int32_t> fill(h.cn_ptr.begin(), h.cn_ptr.end() - 1);
  for (int32_t t = 0; t < coarse.n_tris; ++t)
    for (int v = 0; v < 3; ++v) h.cn_tri[fill[coarse.tri[3 * t + v]]++] = (t << 2) | v;

  // boundary sets
  std::vector<uint8_t> isdir(nf, 0);
  for (size_t e = 0; e < h.fine.btag.size(); ++e)
    if (h.fine.btag[e] == 1) isdir[h.fine.bedge[2 * e]] = isdir[h.fine.bedge[2 * e + 1]] = 1;
  h.dir_index.assign(nf, -1);
  h.dir_nodes.clear();
  for (int32_t i = 0; i < nf; ++i)
    if (isdir[i]) {
      h.dir_index[i] = (int32_t)h.dir_nodes.size();
      h.dir_nodes.push_back(i);
    }
  h.nat_c.assign(nc, 0);
  for (size_t e = 0; e < coarse.btag.size(); ++e)
    if (coarse.btag[e] == 2) h.nat_c[coarse.bedge[2 * e]] = h.nat_c[coarse.bedge[2 * e + 1]] = 1;
  h.n_nat_c = 0;
  for (int32_t i = 0; i < nc; ++i) h.n_nat_c += h.nat_c[i];
  return "";
}

}  // namespace cgp
