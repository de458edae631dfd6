// Host plan of the s-step coarse PCG: tiles, their depth-s neighbourhoods
// and the local ELL blocks of the matrix powers.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <string>
#include <vector>

#include "capcg.hpp"

namespace cgp {
namespace {

// Breadth-first layers around `own` up to distance s.  mark/stamp: a visited
// array reused across calls.  Returns the nodes in layer order (own first)
// and the cumulative layer counts.
void layers(const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col,
            const std::vector<int32_t>& own, int s, std::vector<int32_t>& mark, int32_t stamp,
            std::vector<int32_t>& out, std::vector<int32_t>& cum) {
  out.assign(own.begin(), own.end());
  cum.assign(1, (int32_t)out.size());
  for (int32_t v : own) mark[v] = stamp;
  size_t beg = 0;
  for (int d = 1; d <= s; ++d) {
    const size_t end = out.size();
    for (size_t q = beg; q < end; ++q) {
      const int32_t v = out[q];
      for (int32_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
        const int32_t j = col[k];
        if (mark[j] != stamp) {
          mark[j] = stamp;
          out.push_back(j);
        }
      }
    }
    beg = end;
    cum.push_back((int32_t)out.size());
  }
}

struct Splitter {
  const std::vector<int32_t>& rowptr;
  const std::vector<int32_t>& col;
  const double* xy;
  int s, own_max, ext_max, ell_max, width;
  std::vector<int32_t> mark;
  int32_t stamp = 0;
  std::vector<std::vector<int32_t>> tiles;
  std::string err;

  // the tile's neighbourhood and ELL block fit their capacities
  bool fits(const std::vector<int32_t>& own) {
    std::vector<int32_t> out, cum;
    layers(rowptr, col, own, s, mark, ++stamp, out, cum);
    return (int64_t)out.size() <= ext_max && (int64_t)cum[s - 1] * width <= ell_max;
  }

  // Cuts `nodes` into `parts` tiles by recursive coordinate bisection (the
  // longer side of the bounding box, at the proportional order statistic);
  // a tile over either capacity is halved again.
  void run(std::vector<int32_t> nodes, int parts) {
    if (!err.empty() || nodes.empty()) return;
    if (parts <= 1) {
      if ((int)nodes.size() <= own_max && fits(nodes)) {
        std::sort(nodes.begin(), nodes.end());
        tiles.push_back(std::move(nodes));
        return;
      }
      if (nodes.size() == 1) {
        err = "a coarse node's depth-s neighbourhood exceeds the tile capacity";
        return;
      }
      parts = 2;
    }
    double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
    for (int32_t v : nodes)
      for (int a = 0; a < 2; ++a) {
        lo[a] = std::min(lo[a], xy[2 * v + a]);
        hi[a] = std::max(hi[a], xy[2 * v + a]);
      }
    const int ax = (hi[0] - lo[0]) >= (hi[1] - lo[1]) ? 0 : 1;
    const int p1 = parts / 2;
    size_t mid = (size_t)((double)nodes.size() * p1 / parts + 0.5);
    mid = std::min(std::max<size_t>(mid, 1), nodes.size() - 1);
    // ties broken by node index so the plan does not depend on the library's sort
    std::nth_element(nodes.begin(), nodes.begin() + mid, nodes.end(), [&](int32_t u, int32_t v) {
      const double cu = xy[2 * u + ax], cv = xy[2 * v + ax];
      return cu < cv || (cu == cv && u < v);
    });
    std::vector<int32_t> left(nodes.begin(), nodes.begin() + mid);
    std::vector<int32_t> right(nodes.begin() + mid, nodes.end());
    std::vector<int32_t>().swap(nodes);
    run(std::move(left), p1);
    run(std::move(right), parts - p1);
  }
};

}  // namespace

std::string ca_plan(int32_t n, const std::vector<int32_t>& rowptr,
                    const std::vector<int32_t>& col, const double* xy, int s, int own_max,
                    int ext_max, int ell_max, CaPlan& p) {
  if (n <= 0 || (int64_t)rowptr.size() != (int64_t)n + 1) return "bad graph";
  if (s < 1 || own_max < 1 || ext_max < own_max || ext_max > 65535) return "bad tile limits";
  int width = 1;
  for (int32_t i = 0; i < n; ++i) width = std::max(width, rowptr[i + 1] - rowptr[i]);
  Splitter sp{rowptr, col, xy, s, own_max, ext_max, ell_max, width, std::vector<int32_t>(n, 0)};
  {
    std::vector<int32_t> all(n);
    for (int32_t i = 0; i < n; ++i) all[i] = i;
    sp.run(std::move(all), (n + own_max - 1) / own_max);
  }
  if (!sp.err.empty()) return sp.err;

  p = CaPlan{};
  p.s = s;
  p.ntiles = (int)sp.tiles.size();
  p.ntiles_pad = (p.ntiles + 63) / 64 * 64;
  p.perm.resize(n);
  std::vector<int32_t> inv(n);
  p.own_off.assign(1, 0);
  for (const auto& t : sp.tiles) {
    for (size_t q = 0; q < t.size(); ++q) {
      inv[t[q]] = p.own_off.back() + (int32_t)q;
      p.perm[inv[t[q]]] = t[q];
    }
    p.own_off.push_back(p.own_off.back() + (int32_t)t.size());
    p.max_own = std::max(p.max_own, (int)t.size());
  }

  p.width = width;

  std::vector<int32_t> mark(n, 0), loc(n, -1), out, cum;
  p.ext_off.assign(1, 0);
  p.ell_off.assign(1, 0);
  for (int t = 0; t < p.ntiles; ++t) {
    layers(rowptr, col, sp.tiles[t], s, mark, t + 1, out, cum);
    // internal numbering; each distance class in ascending internal order
    for (int32_t& v : out) v = inv[v];
    for (int d = 1; d <= s; ++d) std::sort(out.begin() + cum[d - 1], out.begin() + cum[d]);
    for (size_t q = 0; q < out.size(); ++q) loc[out[q]] = (int32_t)q;
    p.ext.insert(p.ext.end(), out.begin(), out.end());
    p.ext_off.push_back((int32_t)p.ext.size());
    p.layer.insert(p.layer.end(), cum.begin(), cum.end());
    p.max_ext = std::max(p.max_ext, (int)out.size());
    const int32_t rows = cum[s - 1];
    const size_t base = p.ell_col.size();
    if (base + (size_t)width * rows > (size_t)INT32_MAX) return "plan too large (32-bit ELL offsets)";
    p.ell_col.resize(base + (size_t)width * rows);
    p.ell_slot.resize(base + (size_t)width * rows);
    for (int32_t r = 0; r < rows; ++r) {
      const int32_t e = p.perm[out[r]];
      int k = 0;
      for (int32_t q = rowptr[e]; q < rowptr[e + 1]; ++q, ++k) {
        p.ell_col[base + (size_t)k * rows + r] = (uint16_t)loc[inv[col[q]]];
        p.ell_slot[base + (size_t)k * rows + r] = q;
      }
      for (; k < width; ++k) {
        p.ell_col[base + (size_t)k * rows + r] = (uint16_t)r;
        p.ell_slot[base + (size_t)k * rows + r] = -1;
      }
    }
    p.ell_off.push_back((int32_t)p.ell_col.size());
    for (int32_t v : out) loc[v] = -1;
  }
  return ca_check(n, rowptr, col, p, own_max, ext_max, ell_max);
}

std::string ca_check(int32_t n, const std::vector<int32_t>& rowptr,
                     const std::vector<int32_t>& col, const CaPlan& p, int own_max,
                     int ext_max, int ell_max) {
  const int s = p.s;
  if (s < 1 || p.ntiles < 1 || p.ntiles_pad < p.ntiles || p.ntiles_pad % 64) return "tile count";
  if ((int64_t)p.perm.size() != n || (int64_t)p.own_off.size() != p.ntiles + 1 ||
      (int64_t)p.ext_off.size() != p.ntiles + 1 || (int64_t)p.ell_off.size() != p.ntiles + 1 ||
      (int64_t)p.layer.size() != (int64_t)p.ntiles * (s + 1))
    return "array sizes";
  std::vector<int32_t> seen(n, 0);
  for (int32_t i = 0; i < n; ++i) {
    if (p.perm[i] < 0 || p.perm[i] >= n || seen[p.perm[i]]++) return "perm is not a permutation";
  }
  std::vector<int32_t> inv(n);
  for (int32_t i = 0; i < n; ++i) inv[p.perm[i]] = i;
  if (p.own_off[0] != 0 || p.own_off[p.ntiles] != n) return "own ranges";
  std::vector<int32_t> dist(n, -1), loc(n, -1);
  for (int t = 0; t < p.ntiles; ++t) {
    const int32_t o0 = p.own_off[t], no = p.own_off[t + 1] - o0;
    const int32_t e0 = p.ext_off[t], ne = p.ext_off[t + 1] - e0;
    const int32_t* lay = &p.layer[(size_t)t * (s + 1)];
    if (no < 1 || no > own_max || ne > ext_max || ne > 65535) return "tile size";
    if (lay[0] != no || lay[s] != ne) return "layer bounds";
    for (int d = 1; d <= s; ++d)
      if (lay[d] < lay[d - 1]) return "layer order";
    for (int32_t q = 0; q < ne; ++q) {
      const int32_t v = p.ext[e0 + q];
      if (v < 0 || v >= n || loc[v] >= 0) return "neighbourhood entry";
      loc[v] = q;
      if (q < no && v != o0 + q) return "own nodes are not the tile's range";
    }
    // distances by breadth-first search from the own nodes must match the layers
    std::vector<int32_t> frontier;
    for (int32_t q = 0; q < no; ++q) {
      dist[o0 + q] = 0;
      frontier.push_back(o0 + q);
    }
    std::vector<int32_t> touched(frontier);
    for (int d = 1; d <= s; ++d) {
      std::vector<int32_t> next;
      for (int32_t v : frontier) {
        const int32_t e = p.perm[v];
        for (int32_t k = rowptr[e]; k < rowptr[e + 1]; ++k) {
          const int32_t j = inv[col[k]];
          if (dist[j] < 0) {
            dist[j] = d;
            next.push_back(j);
            touched.push_back(j);
          }
        }
      }
      frontier.swap(next);
    }
    if ((int32_t)touched.size() != ne) return "neighbourhood size";
    for (int32_t v : touched) {
      const int32_t q = loc[v];
      if (q < 0) return "node missing from the neighbourhood";
      const int d = dist[v];
      if (q >= lay[d] || (d > 0 && q < lay[d - 1])) return "node in the wrong layer";
    }
    const int32_t rows = lay[s - 1];
    if ((int64_t)p.width * rows > ell_max) return "ELL block over capacity";
    if ((int64_t)p.ell_off[t + 1] - p.ell_off[t] != (int64_t)p.width * rows) return "ELL block size";
    for (int32_t r = 0; r < rows; ++r) {
      const int32_t e = p.perm[p.ext[e0 + r]];
      const int32_t len = rowptr[e + 1] - rowptr[e];
      if (len > p.width) return "ELL width";
      for (int k = 0; k < p.width; ++k) {
        const size_t at = (size_t)p.ell_off[t] + (size_t)k * rows + r;
        const int32_t lc = p.ell_col[at], sl = p.ell_slot[at];
        if (lc >= ne) return "ELL column out of the neighbourhood";
        if (k < len) {
          if (sl != rowptr[e] + k || p.ext[e0 + lc] != inv[col[sl]]) return "ELL entry";
        } else if (sl != -1 || lc != r) {
          return "ELL padding";
        }
      }
    }
    for (int32_t v : touched) dist[v] = -1;
    for (int32_t q = 0; q < ne; ++q) loc[p.ext[e0 + q]] = -1;
  }
  if ((size_t)p.ell_off[p.ntiles] != p.ell_col.size() || p.ell_col.size() != p.ell_slot.size())
    return "ELL arrays";
  return "";
}

}  // namespace cgp
