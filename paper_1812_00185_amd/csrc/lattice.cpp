// Lattice layout of the fine mesh (host set-up); see lattice.hpp.
#include "lattice.hpp"

#include <algorithm>
#include <unordered_map>

#include "mesh.hpp"
#include "momlat.hpp"

namespace cgp {

LatDev Lattice::host_view() const {
  LatDev d{};
  d.m = m;
  d.nI = nI;
  d.nT = nT;
  d.nE = nE;
  d.nV = nV;
  d.EB = EB;
  d.VB = VB;
  d.tri_v = tri_v.data();
  d.tri_e = tri_e.data();
  d.edge_v = edge_v.data();
  d.edge_t = edge_t.data();
  d.af = af.data();
  d.ldir = ldir.data();
  d.lat_of = lat_of.data();
  d.vw = vw;
  d.vcol = vcol.data();
  d.erec = erec.empty() ? nullptr : erec.data();
  return d;
}

std::string build_lattice(const Hierarchy& h, Lattice& L) {
  L = Lattice{};
  const Mesh& c = h.coarse;
  const int32_t m = 1 << h.levels;
  L.m = m;
  L.nI = (m - 1) * (m - 2) / 2;
  L.nT = c.n_tris;
  L.nV = c.n_nodes;
  L.tri_v = c.tri;
  L.tri_e.assign(3 * (size_t)L.nT, 0);
  std::unordered_map<int64_t, int32_t> eid;
  eid.reserve(3 * (size_t)L.nT);
  for (int32_t T = 0; T < L.nT; ++T)
    for (int j = 0; j < 3; ++j) {
      const int32_t a = c.tri[3 * T + j], b = c.tri[3 * T + (j + 1) % 3];
      const int32_t lo = std::min(a, b), hi = std::max(a, b);
      const int64_t key = (int64_t)lo * L.nV + hi;
      auto it = eid.find(key);
      int32_t E;
      if (it == eid.end()) {
        E = L.nE++;
        eid.emplace(key, E);
        L.edge_v.push_back(lo);
        L.edge_v.push_back(hi);
        L.edge_t.push_back((T << 2) | j);
        L.edge_t.push_back(-1);
      } else {
        E = it->second;
        if (L.edge_t[2 * E + 1] != -1) return "lattice: an edge of more than two triangles";
        L.edge_t[2 * E + 1] = (T << 2) | j;
      }
      L.tri_e[3 * T + j] = (E << 1) | (a == hi ? 1 : 0);
    }
  L.EB = L.nT * L.nI;
  L.VB = L.EB + L.nE * (m - 1);
  const int64_t N = (int64_t)L.VB + L.nV;
  if (N != h.fine.n_nodes) return "lattice: node count differs from the fine mesh";
  L.af.resize(L.nT);
  const double scale = 1.0 / ((double)m * (double)m);  // 4^k
  for (int32_t T = 0; T < L.nT; ++T) {
    const double* p0 = &c.xy[2 * c.tri[3 * T]];
    const double* p1 = &c.xy[2 * c.tri[3 * T + 1]];
    const double* p2 = &c.xy[2 * c.tri[3 * T + 2]];
    const double area = 0.5 * ((p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]));
    L.af[T] = area * scale;
  }
  const LatDev v = L.host_view();  // the index map reads tri_v, tri_e only
  L.lat_of.assign(N, -1);
  std::vector<uint8_t> seen(N, 0);
  for (int32_t i = 0; i < (int32_t)N; ++i) {
    int32_t l;
    if (i < L.nV) {
      l = L.VB + i;
    } else {
      const int32_t T = h.pcode[2 * (size_t)i];
      const int32_t a = h.pcode[2 * (size_t)i + 1] & 0xffff, b = h.pcode[2 * (size_t)i + 1] >> 16;
      if (T < 0 || T >= L.nT || a < 0 || b < 0 || a + b > m)
        return "lattice: prolongation code out of range";
      l = lat_index(v, T, a, b);
    }
    if (l < 0 || l >= N || seen[l]) return "lattice: node map is not a permutation";
    seen[l] = 1;
    L.lat_of[i] = l;
  }
  L.node_of.assign(N, 0);
  for (int32_t i = 0; i < (int32_t)N; ++i) L.node_of[L.lat_of[i]] = i;
  L.ldir.assign(N, 0);
  for (int32_t i = 0; i < (int32_t)N; ++i)
    if (h.dir_index[i] >= 0) L.ldir[L.lat_of[i]] = 1;
  for (int32_t l = 0; l < L.EB; ++l)
    if (L.ldir[l]) return "lattice: Dirichlet node inside a coarse triangle";
  // coarse-vertex rows (mesh nodes 0 .. nV-1): diagonal first, then the rest
  // of the CSR row in order
  const Graph& g = h.gf;
  L.vw = 1;
  for (int32_t v = 0; v < L.nV; ++v) L.vw = std::max(L.vw, g.rowptr[v + 1] - g.rowptr[v]);
  L.vcol.assign((size_t)L.vw * L.nV, 0);
  L.vpos.assign((size_t)L.vw * L.nV, -1);
  for (int32_t v = 0; v < L.nV; ++v) {
    int32_t k = 1;
    bool diag = false;
    for (int32_t s = 0; s < L.vw; ++s) L.vcol[(size_t)s * L.nV + v] = L.VB + v;
    for (int32_t s = g.rowptr[v]; s < g.rowptr[v + 1]; ++s) {
      const int32_t c = g.col[s];
      if (c < 0 || c >= (int32_t)N) return "lattice: vertex row column out of range";
      const int32_t slot = c == v && !diag ? 0 : k++;
      if (c == v) diag = true;
      if (slot >= L.vw) return "lattice: vertex row without its diagonal";
      L.vcol[(size_t)slot * L.nV + v] = L.lat_of[c];
      L.vpos[(size_t)slot * L.nV + v] = s;
    }
    if (!diag) return "lattice: vertex row without its diagonal";
  }
  // the coarse edges' records (from the tables above)
  std::vector<LatEdgeRec> erec(L.nE);
  const LatDev tv = L.host_view();
  if (!lat_dispatch(m, [&](auto lat) {
        constexpr int M = decltype(lat)::kM;
        for (int32_t E = 0; E < L.nE; ++E) erec[E] = Lat<M>::edge_record(tv, E);
      }))
    return "lattice: unsupported lattice size";
  L.erec = std::move(erec);
  return "";
}

void build_mom_slots(const Hierarchy& h, Lattice& L) {
  const Graph& g = h.gf;
  const int32_t N = (int32_t)L.lat_of.size();
  L.mslot.assign(8 * (size_t)N, kNoSlot);
  L.mom_ok = false;
  const LatDev v = L.host_view();
  bool ok = true;
  const bool known = lat_dispatch(v.m, [&](auto lat) {
    constexpr int M = decltype(lat)::kM;
    for (int32_t i = L.nV; i < N && ok; ++i) {
      const int32_t l = L.lat_of[i];
      if (l >= L.VB) {
        ok = false;
        break;
      }
      int32_t pt[6];
      mom_dirs<M>(v, l, pt);
      const int32_t beg = g.rowptr[i], end = g.rowptr[i + 1];
      if (end - beg > 7 || g.col[beg] != i) {  // the kernel stages 7 values per row
        ok = false;
        break;
      }
      std::vector<uint8_t> hit(end - beg, 0);
      int present = 0;
      for (int d = 0; d < 6; ++d) {
        if (pt[d] < 0) continue;
        if (pt[d] >= N) {
          ok = false;
          break;
        }
        ++present;
        const int32_t j = L.node_of[pt[d]];
        int32_t s = beg + 1;
        while (s < end && g.col[s] != j) ++s;
        if (s == end || hit[s - beg]) {
          ok = false;
          break;
        }
        hit[s - beg] = 1;
        L.mslot[8 * (size_t)i + d] = (uint8_t)(s - beg);
      }
      if (ok && present != end - beg - 1) ok = false;
    }
  });
  L.mom_ok = known && ok;
}

}  // namespace cgp
