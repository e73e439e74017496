// Width-set planner (Sec. 2, finding the width set).  Readings of the
// recipe, shared with its statement in the header:
//  * the contraction tree follows an elimination order of vertices;
//    eliminating v leaves a tensor over its scope S(v), the neighbours of v
//    not yet eliminated with fill edges included, so the width of an order
//    is max |S(v)|;
//  * fixing the spins of W removes W and its edges; the tree keeps pi, so
//    the order of R is pi with the W vertices skipped;
//  * pi is greedy min-fill (ties: fewest current neighbours, smallest key);
//  * the sliced index is the vertex in the most scopes of the maximum size
//    (ties: larger degree, smallest key); the bound holds at width <= w_u;
//  * indices go back from W in ascending key order;
//  * with regreedy the tree is rebuilt rather than kept: after every pick
//    and for every re-adding test the min-fill order of the graph induced
//    on R replaces pi restricted to R.
// Graph rows are bitsets, so an elimination costs |S(v)| row operations.
#include "plan.h"

#include <algorithm>
#include <cstdio>

namespace tnvan {
namespace {

using Row = uint64_t;

struct Bits {
  int32_t n = 0, words = 0;
  std::vector<Row> b;   // n rows of `words` words
  Bits(int32_t n_) : n(n_), words((n_ + 63) / 64), b((size_t)n_ * ((n_ + 63) / 64), 0) {}
  Row *row(int32_t v) { return b.data() + (size_t)v * words; }
  const Row *row(int32_t v) const { return b.data() + (size_t)v * words; }
};

inline void set_bit(Row *r, int32_t i) { r[i >> 6] |= Row(1) << (i & 63); }
inline void clear_bit(Row *r, int32_t i) { r[i >> 6] &= ~(Row(1) << (i & 63)); }
inline bool test_bit(const Row *r, int32_t i) { return (r[i >> 6] >> (i & 63)) & 1; }

int32_t popcount(const Row *r, int32_t words) {
  int32_t c = 0;
  for (int32_t w = 0; w < words; ++w) c += __builtin_popcountll(r[w]);
  return c;
}

// calls f(i) for every set bit of r, ascending
template <class F>
void for_bits(const Row *r, int32_t words, F &&f) {
  for (int32_t w = 0; w < words; ++w)
    for (Row x = r[w]; x; x &= x - 1) f(w * 64 + __builtin_ctzll(x));
}

// missing edges among the current neighbours of v
int64_t fill_of(const Bits &g, int32_t v) {
  const Row *rv = g.row(v);
  int64_t f = 0;
  for_bits(rv, g.words, [&](int32_t a) {
    const Row *ra = g.row(a);
    int32_t c = 0;
    for (int32_t w = 0; w < g.words; ++w) c += __builtin_popcountll(rv[w] & ~ra[w]);
    f += c - 1;   // a itself is in N(v) and not in N(a)
  });
  return f / 2;
}

// greedy min-fill order of the graph induced on the vertices not marked in
// `out` (none marked: all of them)
std::vector<int32_t> min_fill(const Bits &g0, const std::vector<int32_t> &key,
                              const std::vector<char> &out) {
  Bits g = g0;
  const int32_t n = g.n, W = g.words;
  std::vector<Row> keep(W, 0);
  std::vector<char> alive(n, 0);
  int32_t m = 0;
  for (int32_t v = 0; v < n; ++v)
    if (!out[v]) { set_bit(keep.data(), v); alive[v] = 1; ++m; }
  for (int32_t v = 0; v < n; ++v) {
    Row *r = g.row(v);
    if (alive[v])
      for (int32_t w = 0; w < W; ++w) r[w] &= keep[w];
    else
      std::fill(r, r + W, Row(0));
  }
  std::vector<int64_t> fill(n, 0);
  std::vector<int32_t> deg(n, 0);
  for (int32_t v = 0; v < n; ++v) {
    if (!alive[v]) continue;
    fill[v] = fill_of(g, v);
    deg[v] = popcount(g.row(v), W);
  }
  std::vector<int32_t> order;
  order.reserve(m);
  std::vector<Row> S(W), dirty(W);
  for (int32_t t = 0; t < m; ++t) {
    int32_t best = -1;
    for (int32_t u = 0; u < n; ++u) {
      if (!alive[u]) continue;
      if (best < 0 || fill[u] < fill[best] ||
          (fill[u] == fill[best] && (deg[u] < deg[best] ||
                                     (deg[u] == deg[best] && key[u] < key[best]))))
        best = u;
    }
    const int32_t v = best;
    order.push_back(v);
    alive[v] = 0;
    std::copy(g.row(v), g.row(v) + W, S.begin());
    std::copy(S.begin(), S.end(), dirty.begin());
    for_bits(S.data(), W, [&](int32_t a) {
      Row *ra = g.row(a);
      clear_bit(ra, v);
      for (int32_t w = 0; w < W; ++w) ra[w] |= S[w];
      clear_bit(ra, a);
    });
    // fills change for S and for every vertex with a neighbour in S
    for_bits(S.data(), W, [&](int32_t a) {
      const Row *ra = g.row(a);
      for (int32_t w = 0; w < W; ++w) dirty[w] |= ra[w];
    });
    std::fill(g.row(v), g.row(v) + W, Row(0));
    for_bits(dirty.data(), W, [&](int32_t u) {
      if (!alive[u]) return;
      fill[u] = fill_of(g, u);
      deg[u] = popcount(g.row(u), W);
    });
  }
  return order;
}

// Eliminates `order` (pi without the vertices marked in `out`) on a copy of
// the graph induced on it.  Returns the width; with counts, adds 1 to
// counts[u] for every u of every scope of size `count_at`.
int32_t eliminate(const Bits &g0, const std::vector<int32_t> &pi, const std::vector<char> &out,
                  std::vector<Row> &rows, std::vector<Row> &alive, int32_t count_at = -1,
                  std::vector<int32_t> *counts = nullptr) {
  const int32_t n = g0.n, W = g0.words;
  std::fill(alive.begin(), alive.end(), Row(0));
  for (int32_t v = 0; v < n; ++v)
    if (!out[v]) set_bit(alive.data(), v);
  rows = g0.b;
  int32_t width = 0;
  std::vector<Row> S(W);
  for (int32_t v : pi) {
    if (out[v]) continue;
    clear_bit(alive.data(), v);
    const Row *rv = rows.data() + (size_t)v * W;
    int32_t s = 0;
    for (int32_t w = 0; w < W; ++w) {
      S[w] = rv[w] & alive[w];
      s += __builtin_popcountll(S[w]);
    }
    width = std::max(width, s);
    if (counts && s == count_at) for_bits(S.data(), W, [&](int32_t u) { ++(*counts)[u]; });
    for_bits(S.data(), W, [&](int32_t a) {
      Row *ra = rows.data() + (size_t)a * W;
      for (int32_t w = 0; w < W; ++w) ra[w] |= S[w];
    });
  }
  return width;
}

}  // namespace

tnvan_status plan_width_set(int32_t n, const std::vector<int32_t> &ei,
                            const std::vector<int32_t> &ej, int32_t w_u,
                            const std::vector<int32_t> &key_in, bool regreedy,
                            PlanResult &res, std::string &msg) {
  char buf[160];
  auto bad = [&](const char *m) { msg = m; return TNVAN_E_INVALID; };
  if (n <= 0 || n > kPlanMaxSpins) {
    std::snprintf(buf, sizeof buf, "n_spins %d out of range 1..%d", n, kPlanMaxSpins);
    return bad(buf);
  }
  if (w_u < 1) return bad("the width bound must be at least 1");
  if (ei.size() != ej.size()) return bad("bad edge arrays");
  std::vector<int32_t> key(n);
  if (key_in.empty()) {
    for (int32_t v = 0; v < n; ++v) key[v] = v;
  } else {
    if ((int32_t)key_in.size() != n) return bad("key must have n entries");
    std::vector<char> seen(n, 0);
    for (int32_t v = 0; v < n; ++v) {
      const int32_t k = key_in[v];
      if (k < 0 || k >= n || seen[k]) return bad("key must be a permutation of 0..n-1");
      seen[k] = 1;
      key[v] = k;
    }
  }
  Bits g(n);
  std::vector<int32_t> deg(n, 0);
  for (size_t e = 0; e < ei.size(); ++e) {
    const int32_t a = ei[e], b = ej[e];
    if (a < 0 || a >= n || b < 0 || b >= n) return bad("edge endpoint out of range");
    if (a == b) return bad("self-loop");
    if (!test_bit(g.row(a), b)) { ++deg[a]; ++deg[b]; }
    set_bit(g.row(a), b);
    set_bit(g.row(b), a);
  }
  std::vector<char> inW(n, 0);
  res.pi = min_fill(g, key, inW);
  std::vector<Row> rows, alive(g.words);
  std::vector<int32_t> counts(n);
  // the order of R: pi without W, or (regreedy) min-fill run again on R
  auto order_of = [&]() {
    if (regreedy) return min_fill(g, key, inW);
    std::vector<int32_t> o;
    for (int32_t v : res.pi)
      if (!inW[v]) o.push_back(v);
    return o;
  };
  // dynamic slicing
  for (;;) {
    const std::vector<int32_t> o = order_of();
    const int32_t w = eliminate(g, o, inW, rows, alive);
    if (w <= w_u) break;
    std::fill(counts.begin(), counts.end(), 0);
    eliminate(g, o, inW, rows, alive, w, &counts);
    int32_t pick = -1;
    for (int32_t u = 0; u < n; ++u) {
      if (!counts[u]) continue;
      if (pick < 0 || counts[u] > counts[pick] ||
          (counts[u] == counts[pick] && (deg[u] > deg[pick] ||
                                         (deg[u] == deg[pick] && key[u] < key[pick]))))
        pick = u;
    }
    inW[pick] = 1;
  }
  // indices back from W, ascending key
  std::vector<int32_t> byk;
  for (int32_t v = 0; v < n; ++v)
    if (inW[v]) byk.push_back(v);
  std::sort(byk.begin(), byk.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  for (int32_t v : byk) {
    inW[v] = 0;
    if (eliminate(g, order_of(), inW, rows, alive) > w_u) inW[v] = 1;
  }
  res.W.clear();
  for (int32_t v = 0; v < n; ++v)
    if (inW[v]) res.W.push_back(v);
  res.order = order_of();
  res.width = eliminate(g, res.order, inW, rows, alive);
  return TNVAN_OK;
}

}  // namespace tnvan
