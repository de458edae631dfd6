// Host-side mesh hierarchy and index structures of the CGP library.
//
// The fine mesh is `levels` uniform 4:1 refinements of the coarse (Poisson)
// mesh (Sect. 2.2).  Everything here is integer/index work done once at
// set-up; the floating-point operators are assembled on the GPU from the
// structures built here.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace cgp {

struct Mesh {
  int32_t n_nodes = 0;
  int32_t n_tris = 0;
  std::vector<double> xy;      // [2 n] interleaved
  std::vector<int32_t> tri;    // [3 T] counter-clockwise
  std::vector<int32_t> bedge;  // [2 B]
  std::vector<int32_t> btag;   // [B]
};

// CSR node graph of a P1 mesh with the diagonal slot first in every row and
// the off-diagonal slots sorted by column.  For an off-diagonal slot (i, j)
// the "sides" are the third vertices of the (one or two) triangles that share
// edge ij: side[2 s] is k with (i, j, k) counter-clockwise, side[2 s + 1] is k
// with (i, k, j) counter-clockwise; -1 where the edge is a boundary edge.
// Diagonal slots carry -1, -1.  Every triangle incident to i appears as two
// sides in row i (once from each of its other two vertices).
struct Graph {
  std::vector<int32_t> rowptr;  // [n + 1]
  std::vector<int32_t> col;     // [nnz]
  std::vector<int32_t> side;    // [2 nnz]
  // row tiles for the LDS-staged SpMV: tile t holds rows [tile[t], tile[t+1]),
  // at most kTileRows rows and kTileNnz nonzeros
  std::vector<int32_t> tile;
  int64_t nnz() const { return (int64_t)col.size(); }
  int32_t ntiles() const { return (int32_t)tile.size() - 1; }
};

constexpr int kTileRows = 256;
constexpr int kTileNnz = 2560;

struct Hierarchy {
  int levels = 0;
  Mesh coarse;
  Mesh fine;
  Graph gc, gf;
  // prolongation code of every fine node: the coarse triangle T holding it and
  // its barycentric coordinates there as integers over 2^levels:
  // pcode[2 i] = T, pcode[2 i + 1] = n1 | (n2 << 16), n0 = 2^levels - n1 - n2
  // (weights of T's vertices 0, 1, 2).
  std::vector<int32_t> pcode;
  // coarse node -> incident coarse triangles, entries (T << 2) | local vertex
  std::vector<int32_t> cn_ptr, cn_tri;
  std::vector<int32_t> dir_nodes;   // sorted fine velocity-Dirichlet nodes
  std::vector<int32_t> dir_index;   // [N_f] position in dir_nodes or -1
  std::vector<uint8_t> nat_c;       // [N_c] 1 where phi = 0 (natural boundary)
  int32_t n_nat_c = 0;
};

// Validates the coarse mesh (index range, distinct vertices, positive area,
// every edge shared by at most two consistently oriented triangles, every
// boundary edge tagged exactly once with a known tag).  Returns "" when valid.
std::string validate(const Mesh& m);

// One level of uniform refinement, new nodes appended in first-encounter
// order (build_hierarchy renumbers the finest level).
Mesh refine(const Mesh& m);

Graph build_graph(const Mesh& m);

// Builds the whole hierarchy; returns "" on success, else the reason.
std::string build_hierarchy(const Mesh& coarse, int levels, Hierarchy& h);

}  // namespace cgp
