// Nested-dissection supernodal Cholesky factor of the coarse Poisson matrix
// (host set-up).  See ndchol.hpp for the layout.
#include "ndchol.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <limits>

namespace cgp {

std::string nd_symbolic(int32_t n, const std::vector<int32_t>& rowptr,
                        const std::vector<int32_t>& col, const double* xy,
                        const std::vector<uint8_t>& skip, NdFactor& f) {
  f = NdFactor{};
  f.n = n;
  f.pos.assign(n, -1);
  std::vector<int32_t> nodes;
  for (int32_t i = 0; i < n; ++i)
    if (!skip[i]) nodes.push_back(i);
  if (nodes.empty()) {
    f.fwd_lvl.assign(1, 0);
    f.bwd_lvl.assign(1, 0);
    return "";
  }

  // ---- ordering: recursive coordinate dissection, children before parents
  std::vector<std::vector<int32_t>> cols;
  std::vector<uint8_t> in_b(n, 0);
  std::function<int32_t(std::vector<int32_t>&)> dissect = [&](std::vector<int32_t>& S) -> int32_t {
    if ((int)S.size() <= kNdLeaf) {
      std::sort(S.begin(), S.end());
      cols.push_back(S);
      f.children.emplace_back();
      return (int32_t)cols.size() - 1;
    }
    double lo[2] = {std::numeric_limits<double>::infinity(), std::numeric_limits<double>::infinity()};
    double hi[2] = {-lo[0], -lo[1]};
    for (int32_t v : S)
      for (int a = 0; a < 2; ++a) {
        lo[a] = std::min(lo[a], xy[2 * v + a]);
        hi[a] = std::max(hi[a], xy[2 * v + a]);
      }
    const int ax = (hi[0] - lo[0]) >= (hi[1] - lo[1]) ? 0 : 1;
    std::sort(S.begin(), S.end(), [&](int32_t a, int32_t b) {
      const double ca = xy[2 * a + ax], cb = xy[2 * b + ax];
      return ca < cb || (ca == cb && a < b);
    });
    const size_t h = S.size() / 2;
    for (size_t k = h; k < S.size(); ++k) in_b[S[k]] = 1;
    std::vector<int32_t> sep, A;
    for (size_t k = 0; k < h; ++k) {
      const int32_t v = S[k];
      bool touches = false;
      for (int32_t e = rowptr[v]; e < rowptr[v + 1] && !touches; ++e) touches = in_b[col[e]] != 0;
      (touches ? sep : A).push_back(v);
    }
    for (size_t k = h; k < S.size(); ++k) in_b[S[k]] = 0;
    if (sep.empty()) {  // the halves are not connected: any node separates them
      sep.push_back(A.back());
      A.pop_back();
    }
    std::vector<int32_t> B(S.begin() + h, S.end());
    std::vector<int32_t>().swap(S);
    std::vector<int32_t> ch;
    if (!A.empty()) ch.push_back(dissect(A));
    ch.push_back(dissect(B));
    std::sort(sep.begin(), sep.end());
    cols.push_back(std::move(sep));
    f.children.push_back(std::move(ch));
    return (int32_t)cols.size() - 1;
  };
  dissect(nodes);

  const int32_t nsn = (int32_t)cols.size();
  f.sn.resize(nsn);
  int32_t c0 = 0;
  for (int32_t s = 0; s < nsn; ++s) {
    NdSuper& S = f.sn[s];
    S.c0 = c0;
    S.w = (int32_t)cols[s].size();
    for (int32_t v : cols[s]) {
      f.pos[v] = (int32_t)f.perm.size();
      f.perm.push_back(v);
    }
    c0 += S.w;
    int lev = 0;
    for (int32_t c : f.children[s]) lev = std::max(lev, f.sn[c].level + 1);
    S.level = lev;
    f.height = std::max(f.height, lev + 1);
  }
  f.nfac = c0;

  // ---- below-diagonal structure: R_s = (adj(C_s) u children's R) past C_s
  std::vector<int32_t> mark(f.nfac, -1);
  std::vector<std::vector<int32_t>> R(nsn);
  for (int32_t s = 0; s < nsn; ++s) {
    const NdSuper& S = f.sn[s];
    const int32_t c1 = S.c0 + S.w;
    std::vector<int32_t>& r = R[s];
    for (int32_t j = 0; j < S.w; ++j) {
      const int32_t v = f.perm[S.c0 + j];
      for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
        const int32_t p = f.pos[col[e]];
        if (p >= c1 && mark[p] != s) {
          mark[p] = s;
          r.push_back(p);
        }
      }
    }
    for (int32_t c : f.children[s])
      for (int32_t p : R[c]) {
        if (p < S.c0) return "nested dissection: child row outside its ancestors";
        if (p >= c1 && mark[p] != s) {
          mark[p] = s;
          r.push_back(p);
        }
      }
    std::sort(r.begin(), r.end());
  }

  // ---- offsets, scatter lists of the children's update vectors
  int64_t goff = 0;
  int32_t roff = 0, uoff = 0, gpos = 0;
  for (int32_t s = 0; s < nsn; ++s) {
    NdSuper& S = f.sn[s];
    S.m = (int32_t)R[s].size();
    S.goff = goff;
    S.roff = roff;
    S.uoff = uoff;
    S.gpos = gpos;
    const int32_t fs = S.w + S.m;
    goff += (int64_t)fs * S.w;
    roff += S.m;
    uoff += S.m;
    gpos += fs;
    f.max_w = std::max(f.max_w, S.w);
    f.max_front = std::max(f.max_front, fs);
    f.rows.insert(f.rows.end(), R[s].begin(), R[s].end());
  }
  if (f.max_front > kNdMaxFront)
    return "nested dissection: a front exceeds " + std::to_string(kNdMaxFront) + " rows";
  f.g_entries = goff;
  f.n_upd = uoff;
  f.gptr.assign((size_t)gpos + 1, 0);
  {
    // counts, then fill in (child, entry) order
    for (int32_t s = 0; s < nsn; ++s) {
      const NdSuper& S = f.sn[s];
      const int32_t c1 = S.c0 + S.w;
      for (int32_t c : f.children[s])
        for (int32_t p : R[c]) {
          const int32_t o = p < c1 ? p - S.c0
                                   : S.w + (int32_t)(std::lower_bound(R[s].begin(), R[s].end(), p) -
                                                     R[s].begin());
          ++f.gptr[S.gpos + o + 1];
        }
    }
    for (int32_t i = 0; i < gpos; ++i) f.gptr[i + 1] += f.gptr[i];
    f.gidx.assign(f.gptr[gpos], 0);
    std::vector<int32_t> fill(f.gptr.begin(), f.gptr.end() - 1);
    for (int32_t s = 0; s < nsn; ++s) {
      const NdSuper& S = f.sn[s];
      const int32_t c1 = S.c0 + S.w;
      for (int32_t c : f.children[s]) {
        const NdSuper& Cc = f.sn[c];
        for (int32_t k = 0; k < Cc.m; ++k) {
          const int32_t p = R[c][k];
          const int32_t o = p < c1 ? p - S.c0
                                   : S.w + (int32_t)(std::lower_bound(R[s].begin(), R[s].end(), p) -
                                                     R[s].begin());
          f.gidx[fill[S.gpos + o]++] = Cc.uoff + k;
        }
      }
    }
  }

  // ---- work items by level
  f.fwd_lvl.assign(f.height + 1, 0);
  f.bwd_lvl.assign(f.height + 1, 0);
  for (int32_t L = 0; L < f.height; ++L) {
    f.fwd_lvl[L] = (int32_t)f.fwd.size();
    for (int32_t s = 0; s < nsn; ++s) {
      const NdSuper& S = f.sn[s];
      if (S.level != L) continue;
      for (int32_t lo = 0; lo < S.w + S.m; lo += kNdItemRows)
        f.fwd.push_back(NdItem{s, lo, std::min(lo + kNdItemRows, S.w + S.m)});
    }
  }
  f.fwd_lvl[f.height] = (int32_t)f.fwd.size();
  // backward: root level first; bwd_lvl[q] .. bwd_lvl[q+1] is level height-1-q
  for (int32_t q = 0; q < f.height; ++q) {
    const int32_t L = f.height - 1 - q;
    f.bwd_lvl[q] = (int32_t)f.bwd.size();
    for (int32_t s = 0; s < nsn; ++s) {
      const NdSuper& S = f.sn[s];
      if (S.level != L) continue;
      for (int32_t lo = 0; lo < S.w; lo += kNdItemRows)
        f.bwd.push_back(NdItem{s, lo, std::min(lo + kNdItemRows, S.w)});
    }
  }
  f.bwd_lvl[f.height] = (int32_t)f.bwd.size();
  return "";
}

std::string nd_numeric(const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col,
                       const double* val, NdFactor& f) {
  f.G.assign((size_t)f.g_entries, 0.0);
  f.GT.assign((size_t)f.g_entries, 0.0);
  const int32_t nsn = (int32_t)f.sn.size();
  std::vector<std::vector<double>> upd(nsn);  // Schur updates, m x m lower, row-major
  std::vector<int32_t> fpos(f.nfac, -1);
  std::vector<double> F, D;
  for (int32_t s = 0; s < nsn; ++s) {
    const NdSuper& S = f.sn[s];
    const int32_t w = S.w, m = S.m, fs = w + m;
    const int32_t* R = f.rows.data() + S.roff;
    for (int32_t j = 0; j < w; ++j) fpos[S.c0 + j] = j;
    for (int32_t k = 0; k < m; ++k) fpos[R[k]] = w + k;
    // front: original entries of the columns of s (lower triangle), then the
    // children's updates
    F.assign((size_t)fs * fs, 0.0);
    for (int32_t j = 0; j < w; ++j) {
      const int32_t v = f.perm[S.c0 + j];
      for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
        const int32_t p = f.pos[col[e]];
        if (p < S.c0) continue;  // skipped node, or a column eliminated below
        const int32_t a = fpos[p];
        if (a < j) continue;     // upper triangle: taken from the other row
        F[(size_t)a * fs + j] = val[e];
      }
    }
    for (int32_t c : f.children[s]) {
      const NdSuper& Cc = f.sn[c];
      const int32_t* Rc = f.rows.data() + Cc.roff;
      const std::vector<double>& U = upd[c];
      for (int32_t k1 = 0; k1 < Cc.m; ++k1) {
        const int32_t a1 = fpos[Rc[k1]];
        for (int32_t k2 = 0; k2 <= k1; ++k2) F[(size_t)a1 * fs + fpos[Rc[k2]]] += U[(size_t)k1 * Cc.m + k2];
      }
      std::vector<double>().swap(upd[c]);
    }
    // left-looking Cholesky of the first w columns over all fs rows: L11 and L21
    for (int32_t j = 0; j < w; ++j) {
      const double* Fj = &F[(size_t)j * fs];
      double d = Fj[j];
      for (int32_t k = 0; k < j; ++k) d -= Fj[k] * Fj[k];
      if (!(d > 0.0) || !std::isfinite(d))
        return "coarse factorisation: non-positive pivot (matrix not positive definite)";
      const double ljj = std::sqrt(d);
      F[(size_t)j * fs + j] = ljj;
      for (int32_t i = j + 1; i < fs; ++i) {
        double* Fi = &F[(size_t)i * fs];
        double t = Fi[j];
        for (int32_t k = 0; k < j; ++k) t -= Fi[k] * Fj[k];
        Fi[j] = t / ljj;
      }
    }
    // Schur complement F22 - L21 L21^T for the parent
    if (m > 0) {
      std::vector<double>& U = upd[s];
      U.assign((size_t)m * m, 0.0);
      for (int32_t a = 0; a < m; ++a) {
        const double* La = &F[(size_t)(w + a) * fs];
        for (int32_t b = 0; b <= a; ++b) {
          const double* Lb = &F[(size_t)(w + b) * fs];
          double t = La[w + b];
          for (int32_t k = 0; k < w; ++k) t -= La[k] * Lb[k];
          U[(size_t)a * m + b] = t;
        }
      }
    }
    // D = L11^-1 (lower), row-major
    D.assign((size_t)w * w, 0.0);
    for (int32_t j = 0; j < w; ++j) {
      D[(size_t)j * w + j] = 1.0 / F[(size_t)j * fs + j];
      for (int32_t i = j + 1; i < w; ++i) {
        const double* Li = &F[(size_t)i * fs];
        double t = 0.0;
        for (int32_t k = j; k < i; ++k) t += Li[k] * D[(size_t)k * w + j];
        D[(size_t)i * w + j] = -t / Li[i];
      }
    }
    // G = [D ; L21 D] column-major (ld fs) and G^T column-major (ld w)
    double* G = f.G.data() + S.goff;
    double* GT = f.GT.data() + S.goff;
    for (int32_t o = 0; o < fs; ++o) {
      for (int32_t j = 0; j < w; ++j) {
        double g;
        if (o < w) {
          g = D[(size_t)o * w + j];
        } else {
          const double* Lo = &F[(size_t)o * fs];
          g = 0.0;
          for (int32_t k = j; k < w; ++k) g += Lo[k] * D[(size_t)k * w + j];
        }
        G[o + (size_t)j * fs] = g;
        GT[j + (size_t)o * w] = g;
      }
    }
    for (int32_t j = 0; j < w; ++j) fpos[S.c0 + j] = -1;
    for (int32_t k = 0; k < m; ++k) fpos[R[k]] = -1;
  }
  return "";
}

void nd_solve_host(const NdFactor& f, const double* r, double* z) {
  std::vector<double> Y(f.nfac), X(f.nfac), U(f.n_upd), fc((size_t)f.max_w), v((size_t)f.max_front);
  for (int32_t i = 0; i < f.n; ++i) z[i] = 0.0;
  auto gathered = [&](const NdSuper& S, int32_t o) {
    double t = 0.0;
    for (int32_t q = f.gptr[S.gpos + o]; q < f.gptr[S.gpos + o + 1]; ++q) t += U[f.gidx[q]];
    return t;
  };
  for (const NdItem& it : f.fwd) {
    const NdSuper& S = f.sn[it.sn];
    const int32_t fs = S.w + S.m;
    for (int32_t j = 0; j < S.w; ++j) fc[j] = r[f.perm[S.c0 + j]] + gathered(S, j);
    const double* G = f.G.data() + S.goff;
    const int32_t jmax = it.hi <= S.w ? it.hi : S.w;  // D is lower triangular
    for (int32_t o = it.lo; o < it.hi; ++o) {
      double acc = 0.0;
      for (int32_t j = 0; j < jmax; ++j) acc += G[o + (size_t)j * fs] * fc[j];
      if (o < S.w) Y[S.c0 + o] = acc;
      else U[S.uoff + o - S.w] = gathered(S, o) - acc;
    }
  }
  for (const NdItem& it : f.bwd) {
    const NdSuper& S = f.sn[it.sn];
    const int32_t fs = S.w + S.m;
    for (int32_t o = 0; o < fs; ++o)
      v[o] = o < S.w ? Y[S.c0 + o] : -X[f.rows[S.roff + o - S.w]];
    const double* GT = f.GT.data() + S.goff;
    for (int32_t i = it.lo; i < it.hi; ++i) {
      double acc = 0.0;
      for (int32_t o = it.lo; o < fs; ++o) acc += GT[i + (size_t)o * S.w] * v[o];
      X[S.c0 + i] = acc;
      z[f.perm[S.c0 + i]] = acc;
    }
  }
}

}  // namespace cgp
