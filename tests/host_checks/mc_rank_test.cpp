// Host check of the Monte Carlo kernel's rank table (csrc/mc_rank.hpp, the
// header the library compiles): for random chunks of isovalues -- ties,
// infinities, empty slots, 8 and 16 slots -- the table's search gives every
// value's rank #{q : c_q <= d} over the chunk (empty slots count as +inf),
// perm lists the isovalues in ascending order with ties in their given
// order, and a NaN isovalue is refused.  Built with g++ under ASan/UBSan.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2510_01190_amd/csrc/mc_rank.hpp"

namespace {

int failures = 0;

void check(bool ok, const char* what, int trial) {
  if (!ok) {
    if (failures < 20) std::printf("FAIL %s (trial %d)\n", what, trial);
    ++failures;
  }
}

// The walk the kernel takes over the table (node index i instead of its
// byte offset 4i).
int search(const pdiv::RankTable& t, int slots, float d) {
  int i = 1;
  for (int k = 1; k < slots; k *= 2) i = 2 * i + (d >= t.tree[i] ? 1 : 0);
  return i - slots + (d >= t.tree[0] ? 1 : 0);
}

}  // namespace

int main() {
  std::mt19937 rng(12345);
  std::normal_distribution<float> nd(0.0f, 1.0f);
  const float inf = std::numeric_limits<float>::infinity();
  for (int trial = 0; trial < 20000; ++trial) {
    const int slots = (trial & 1) ? 16 : 8;
    const int kc = 1 + int(rng() % unsigned(slots));
    std::vector<float> c(16, 0.0f);
    for (int q = 0; q < kc; ++q) c[size_t(q)] = nd(rng);
    if (trial % 3 == 0)  // ties
      for (int q = 1; q < kc; q += 2) c[size_t(q)] = c[size_t(q - 1)];
    if (trial % 7 == 0) c[size_t(rng() % unsigned(kc))] = (rng() & 1) ? inf : -inf;
    if (trial % 11 == 0) c[size_t(rng() % unsigned(kc))] = -0.0f;
    pdiv::RankTable t;
    check(pdiv::rank_table(c.data(), kc, slots, &t), "table built", trial);
    // perm: ascending, stable among equal values, a permutation of 0..kc-1
    std::vector<int> order(static_cast<size_t>(kc));
    for (int q = 0; q < kc; ++q) order[size_t(q)] = q;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return c[size_t(a)] < c[size_t(b)]; });
    for (int q = 0; q < kc; ++q) check(t.perm[q] == order[size_t(q)], "perm", trial);
    // ranks of random, tied, boundary and infinite values
    std::vector<float> ds;
    for (int n = 0; n < 24; ++n) ds.push_back(1.5f * nd(rng));
    for (int q = 0; q < kc; ++q) {
      ds.push_back(c[size_t(q)]);
      ds.push_back(std::nextafter(c[size_t(q)], -inf));
    }
    ds.push_back(inf);
    ds.push_back(-inf);
    for (float d : ds) {
      int want = 0;
      for (int q = 0; q < slots; ++q) want += (q < kc ? c[size_t(q)] : inf) <= d ? 1 : 0;
      check(search(t, slots, d) == want, "rank", trial);
    }
    // NaN (which no comparison places) ranks 0 and a NaN isovalue is refused
    check(search(t, slots, std::nanf("")) == 0, "nan rank", trial);
    c[size_t(rng() % unsigned(kc))] = std::nanf("");
    check(!pdiv::rank_table(c.data(), kc, slots, &t), "nan refused", trial);
  }
  pdiv::RankTable t;
  const float one[1] = {0.5f};
  check(!pdiv::rank_table(one, 1, 4, &t), "slots other than 8 or 16 refused", -1);
  check(!pdiv::rank_table(one, 0, 8, &t), "empty chunk refused", -1);
  if (failures == 0) std::printf("ALL PASS\n");
  return failures == 0 ? 0 : 1;
}
