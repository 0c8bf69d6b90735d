// Host side of the Monte Carlo kernel's ranked crossing test: the sorted
// isovalue table the kernel searches.  Plain C++ (no HIP), so that a host
// test can build it as the library does.
#pragma once

#include <limits>

namespace pdiv {

// The isovalues of a chunk of K = 8 or 16 slots in ascending order:
// tree[1..K-1] holds the K-1 smallest in breadth-first order of a complete
// binary search tree (node i's children are 2i and 2i+1; an in-order walk
// visits them sorted), tree[0] the largest; perm[q] is the output plane of
// the q-th smallest.  A vertex divergence d ranks #{q : c_q <= d}: from node
// 1, go to child 2i + (d >= tree[i]) log2 K times, land on i in [K, 2K),
// and add d >= tree[0] to i - K.
struct RankTable {
  float tree[16];
  int perm[16];
};

// The table for a chunk of kc <= slots isovalues c[0..kc) (slots = 8 or 16),
// or false when the chunk holds a NaN (which no ordering places).  Slots past
// kc hold +inf: a vertex ranks above them only at +inf, and their counts are
// not stored.  Equal isovalues keep their order (a stable sort).
inline bool rank_table(const float* c, int kc, int slots, RankTable* rt) {
  if (kc < 1 || kc > slots || (slots != 8 && slots != 16)) return false;
  int idx[16];
  for (int q = 0; q < 16; ++q) {
    if (q < kc && c[q] != c[q]) return false;
    idx[q] = q;
  }
  for (int a = 1; a < kc; ++a) {  // stable insertion sort of the kc values
    const int v = idx[a];
    int b = a;
    for (; b > 0 && c[idx[b - 1]] > c[v]; --b) idx[b] = idx[b - 1];
    idx[b] = v;
  }
  constexpr float kInf = std::numeric_limits<float>::infinity();
  float sorted[16];
  for (int q = 0; q < 16; ++q) {
    sorted[q] = q < kc ? c[idx[q]] : kInf;
    rt->perm[q] = q < kc ? idx[q] : 0;
    rt->tree[q] = kInf;
  }
  // breadth-first placement of sorted[0..slots-2]: an in-order walk of the
  // nodes 1..slots-1
  int next = 0;
  int stack[8], top = 0, node = 1;
  while (top > 0 || node < slots) {
    while (node < slots) {
      stack[top++] = node;
      node *= 2;
    }
    node = stack[--top];
    rt->tree[node] = sorted[next++];
    node = 2 * node + 1;
  }
  rt->tree[0] = sorted[slots - 1];
  return true;
}

}  // namespace pdiv
