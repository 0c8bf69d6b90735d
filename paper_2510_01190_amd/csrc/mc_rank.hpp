// The Monte Carlo kernel's ranked crossing test, the parts that are plain
// C++: the sorted isovalue table the kernel searches (built on the host) and
// the bit-sliced crossing counters (constexpr, so the kernel and a host test
// compile the same functions).
#pragma once

#include <cstdint>
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

// Crossing counts of 32 (cell, isovalue) slots in bit-sliced form: bit j of
// s[b] / t[b] is bit b of slot j's count.  sliced_add2 adds the 0/1 masks
// of two samples to the 4-plane counter s (which holds at most 15: flush
// after at most 7 pairs); sliced_flush adds s into the 16-plane counter t
// (counts up to 65535) and clears s.
struct Sliced {
  uint32_t s[4];
  uint32_t t[16];
};

constexpr void sliced_clear(Sliced& c) {
  for (int b = 0; b < 4; ++b) c.s[b] = 0u;
  for (int b = 0; b < 16; ++b) c.t[b] = 0u;
}

constexpr void sliced_add2(Sliced& c, uint32_t w0, uint32_t w1) {
  const uint32_t x = w0 ^ w1, y = w0 & w1;  // the pair's sum: y x, two bits
  const uint32_t c0 = c.s[0] & x;
  c.s[0] ^= x;
  const uint32_t t1 = c.s[1] ^ y;
  const uint32_t c1 = (c.s[1] & y) | (t1 & c0);
  c.s[1] = t1 ^ c0;
  const uint32_t c2 = c.s[2] & c1;
  c.s[2] ^= c1;
  c.s[3] ^= c2;
}

constexpr void sliced_flush(Sliced& c) {
  uint32_t carry = c.t[0] & c.s[0];
  c.t[0] ^= c.s[0];
  for (int b = 1; b < 4; ++b) {
    const uint32_t u = c.t[b] ^ c.s[b];
    const uint32_t nc = (c.t[b] & c.s[b]) | (u & carry);
    c.t[b] = u ^ carry;
    carry = nc;
  }
  for (int b = 4; b < 16; ++b) {
    const uint32_t nc = c.t[b] & carry;
    c.t[b] ^= carry;
    carry = nc;
  }
  for (int b = 0; b < 4; ++b) c.s[b] = 0u;
}

constexpr uint32_t sliced_count(const Sliced& c, int j) {
  uint32_t n = 0;
  for (int b = 0; b < 16; ++b) n |= ((c.t[b] >> j) & 1u) << b;
  return n;
}

// Crossed isovalues of a cell from its corners' ranks: the bits rmin..rmax-1
// (ranks are at most 16).
constexpr uint32_t crossed_mask(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3) {
  const uint32_t lo01 = r0 < r1 ? r0 : r1, lo23 = r2 < r3 ? r2 : r3;
  const uint32_t hi01 = r0 < r1 ? r1 : r0, hi23 = r2 < r3 ? r3 : r2;
  const uint32_t lo = lo01 < lo23 ? lo01 : lo23, hi = hi01 < hi23 ? hi23 : hi01;
  return ((1u << (hi - lo)) - 1u) << lo;
}

}  // namespace pdiv
