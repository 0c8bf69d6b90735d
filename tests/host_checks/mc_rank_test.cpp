// Host check of the Monte Carlo kernel's ranked crossing test
// (csrc/mc_rank.hpp, the header the library compiles).  Rank table: for
// random chunks of isovalues -- ties, infinities, empty slots, 8 and 16
// slots -- the table's search gives every value's rank #{q : c_q <= d} over
// the chunk (empty slots count as +inf), perm lists the isovalues in
// ascending order with ties in their given order, and a NaN isovalue is
// refused.  Crossed masks: the bits rmin..rmax-1 of every rank quadruple.
// Bit-sliced counters: for random masks, in the two flush patterns the
// kernels use, every slot's count equals the plain count, up to 65535.
// Built with g++ under ASan/UBSan.
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
  // crossed masks of every rank quadruple (ranks 0..16)
  for (uint32_t r0 = 0; r0 <= 16; ++r0)
    for (uint32_t r1 = 0; r1 <= 16; ++r1)
      for (uint32_t r2 = 0; r2 <= 16; r2 += 3)
        for (uint32_t r3 = 0; r3 <= 16; r3 += 5) {
          const uint32_t lo = std::min(std::min(r0, r1), std::min(r2, r3));
          const uint32_t hi = std::max(std::max(r0, r1), std::max(r2, r3));
          uint32_t want = 0;
          for (uint32_t q = 0; q < 16; ++q) want |= (lo <= q && q < hi ? 1u : 0u) << q;
          check(pdiv::crossed_mask(r0, r1, r2, r3) == want, "crossed mask", int(r0 * 17 + r1));
        }
  // bit-sliced counters against plain counts: the vector kernel adds one
  // pair per step and flushes after every 7th, the vertex kernel adds two
  // pairs per step and flushes after every 3rd; a final flush in both
  for (int trial = 0; trial < 400; ++trial) {
    const int n = trial == 0 ? 65535 : 1 + int(rng() % 3000u);
    const bool vertex = trial % 2 == 1;
    const unsigned density = 1u + rng() % 31u;  // bits set with probability density/32
    pdiv::Sliced sl;
    pdiv::sliced_clear(sl);
    std::vector<uint32_t> plain(32, 0);
    std::vector<uint32_t> words;
    for (int smp = 0; smp < n; ++smp) {
      uint32_t w = 0;
      for (int b = 0; b < 32; ++b) w |= (trial == 0 || rng() % 32u < density ? 1u : 0u) << b;
      words.push_back(w);
      for (int b = 0; b < 32; ++b) plain[size_t(b)] += (w >> b) & 1u;
    }
    const int per_step = vertex ? 4 : 2, flush_every = vertex ? 3 : 7;
    int step = 0;
    for (int s0 = 0; s0 < n; s0 += per_step, ++step) {
      for (int p = 0; p < per_step; p += 2) {
        const uint32_t w0 = s0 + p < n ? words[size_t(s0 + p)] : 0u;
        const uint32_t w1 = s0 + p + 1 < n ? words[size_t(s0 + p + 1)] : 0u;
        pdiv::sliced_add2(sl, w0, w1);
      }
      if (step % flush_every == flush_every - 1) pdiv::sliced_flush(sl);
    }
    pdiv::sliced_flush(sl);
    for (int b = 0; b < 32; ++b)
      check(pdiv::sliced_count(sl, b) == plain[size_t(b)], "sliced count", trial);
  }
  pdiv::RankTable t;
  const float one[1] = {0.5f};
  check(!pdiv::rank_table(one, 1, 4, &t), "slots other than 8 or 16 refused", -1);
  check(!pdiv::rank_table(one, 0, 8, &t), "empty chunk refused", -1);
  if (failures == 0) std::printf("ALL PASS\n");
  return failures == 0 ? 0 : 1;
}
