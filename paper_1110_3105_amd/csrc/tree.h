// Host-side index tree (quadtree / octree) with contiguous index ranges.
#pragma once

#include <stdint.h>

#include <vector>

namespace rs {

struct Tree {
  int dim = 0;
  int64_t n = 0;
  int leaf_size = 0;
  int maxdepth = 0;
  std::vector<int64_t> perm;      // tree position i holds caller point perm[i]
  std::vector<double> center;     // 3 per box (unused axes 0)
  std::vector<double> side;
  std::vector<int> depth, parent;
  std::vector<int64_t> begin, end;
  std::vector<int> first_child, nchild;   // children are consecutive (breadth-first ids)
  std::vector<int64_t> icoord;            // 3 per box: integer cell of the box at its depth
  std::vector<std::vector<int>> levels;   // box ids per depth, in tree order
  std::vector<double> coords;             // dim x n, tree order (structure of arrays)

  int nbox() const { return (int)side.size(); }
  bool is_leaf(int b) const { return nchild[b] == 0; }
  void build(int dim, int64_t n, const double *points, int leaf_size);

  Tree() = default;
  Tree(const Tree &) = default;
  Tree(Tree &&) = default;
  Tree &operator=(const Tree &) = default;
  Tree &operator=(Tree &&) = default;
  // The per-point arrays go back to a process-wide cache for the next build (their
  // pages are already mapped: first-touch faults on fresh arrays were most of a build).
  ~Tree();
};

}  // namespace rs

struct rs_tree_s {
  rs::Tree t;
};
