// Host-only checks of the instance compiler and the width-set planner,
// built with AddressSanitizer and UndefinedBehaviorSanitizer (no GPU, no
// HIP): valid programs compile with the expected statistics, malformed
// instances are refused with the expected status, the planner meets its
// bound, and seeded random instances and plans (valid or not) never read or
// write out of bounds.  Exit status 0 when every check holds.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../../include/tnvan.h"
#include "../../paper_2504_12037_amd/csrc/compile.h"
#include "../../paper_2504_12037_amd/csrc/plan.h"

using namespace tnvan;

static int g_fail = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++g_fail;                                                         \
    }                                                                   \
  } while (0)

struct Inst {
  int n = 0;
  std::vector<int32_t> ei, ej, W, order, gp;
  std::vector<double> J, h;
  double beta = 1.0;
  int hidden = 0;
  tnvan_instance c() const {
    tnvan_instance t{};
    t.n_spins = n;
    t.n_edges = (int32_t)ei.size();
    t.edge_i = ei.empty() ? nullptr : ei.data();
    t.edge_j = ej.empty() ? nullptr : ej.data();
    t.J = J.empty() ? nullptr : J.data();
    t.h = h.empty() ? nullptr : h.data();
    t.beta = beta;
    t.n_width = (int32_t)W.size();
    t.width_set = W.empty() ? nullptr : W.data();
    t.n_order = (int32_t)order.size();
    t.order = order.empty() ? nullptr : order.data();
    t.n_groups = gp.empty() ? 0 : (int32_t)gp.size() - 1;
    t.group_ptr = gp.empty() ? nullptr : gp.data();
    t.hidden = hidden;
    return t;
  }
};

// L x L open lattice, W = the given 1-based columns, the rest row by row in
// strips, one group per strip row when rows is set
static Inst lattice(int L, std::vector<int> wcols, bool rows, std::mt19937_64 &rng) {
  Inst I;
  I.n = L * L;
  std::normal_distribution<double> nd;
  for (int r = 0; r < L; ++r)
    for (int c = 0; c + 1 < L; ++c) { I.ei.push_back(r * L + c); I.ej.push_back(r * L + c + 1); }
  for (int r = 0; r + 1 < L; ++r)
    for (int c = 0; c < L; ++c) { I.ei.push_back(r * L + c); I.ej.push_back((r + 1) * L + c); }
  for (size_t e = 0; e < I.ei.size(); ++e) I.J.push_back(nd(rng));
  for (int v = 0; v < I.n; ++v) I.h.push_back(0.1 * nd(rng));
  std::vector<int> isw(L + 1, 0);
  for (int c : wcols) isw[c] = 1;
  for (int r = 0; r < L; ++r)
    for (int c = 1; c <= L; ++c)
      if (isw[c]) I.W.push_back(r * L + c - 1);
  // strips between W columns
  std::vector<std::pair<int, int>> strips;
  int c0 = 1;
  for (int c = 1; c <= L + 1; ++c)
    if (c == L + 1 || isw[c]) {
      if (c > c0) strips.push_back({c0, c - 1});
      c0 = c + 1;
    }
  if (rows) I.gp.push_back(0);
  for (auto &s : strips)
    for (int r = 0; r < L; ++r) {
      for (int c = s.first; c <= s.second; ++c) I.order.push_back(r * L + c - 1);
      if (rows) I.gp.push_back((int32_t)I.order.size());
    }
  return I;
}

// a random graph of degree about d on n vertices with a random W of size m
// and a random order of the rest
static Inst random_graph(int n, int d, int m, std::mt19937_64 &rng) {
  Inst I;
  I.n = n;
  std::vector<std::vector<char>> adj(n, std::vector<char>(n, 0));
  std::uniform_int_distribution<int> U(0, n - 1);
  for (int k = 0; k < n * d / 2; ++k) {
    int a = U(rng), b = U(rng);
    if (a == b) continue;
    if (a > b) std::swap(a, b);
    if (adj[a][b]) continue;
    adj[a][b] = 1;
    I.ei.push_back(a);
    I.ej.push_back(b);
    I.J.push_back(rng() & 1 ? 1.0 : -1.0);
  }
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  std::shuffle(perm.begin(), perm.end(), rng);
  for (int i = 0; i < n; ++i) (i < m ? I.W : I.order).push_back(perm[i]);
  return I;
}

static tnvan_status compile(const Inst &I, int maxw, HostProgram &P, std::string &msg) {
  const tnvan_instance t = I.c();
  return compile_instance(t, maxw, P, msg);
}

int main() {
  std::mt19937_64 rng(12345);
  std::string msg;
  // --- valid programs and their statistics
  {
    HostProgram P;
    Inst I = lattice(4, {2}, true, rng);
    CHECK(compile(I, 14, P, msg) == TNVAN_OK);
    CHECK(P.insts.size() == 1 && P.insts[0].nw == 4 && P.insts[0].nr == 12);
    CHECK(P.insts[0].n_steps == 8 && P.insts[0].max_w == 2);
    Inst I2 = lattice(16, {6, 11}, true, rng);
    CHECK(compile(I2, 14, P, msg) == TNVAN_OK);
    CHECK(P.insts.size() == 2 && P.insts[1].n_steps == 48 && P.insts[1].max_w == 5);
    CHECK(P.cinst.size() == 2 && P.cinst[1].ok == 1 && P.cinst[1].n_chains == 3);
    Inst I3 = lattice(8, {5}, false, rng);
    CHECK(compile(I3, 14, P, msg) == TNVAN_OK);
    // every gather table entry indexes inside its input message
    for (const StepDesc &sd : P.steps)
      for (int k = 0; k < sd.n_in; ++k) {
        const InputDesc &id = P.inputs[sd.in_off + k];
        if (id.gb_off < 0) continue;
        for (int o = 0; o < (1 << sd.w); ++o) CHECK(P.gtab[id.gb_off + o] < (1u << id.nbits));
      }
  }
  // --- malformed instances
  {
    Inst base = lattice(4, {2}, true, rng);
    auto expect = [&](Inst I, tnvan_status want, const char *what) {
      HostProgram P;
      const tnvan_status s = compile(I, 14, P, msg);
      if (s != want) std::fprintf(stderr, "%s: status %d, message %s\n", what, (int)s, msg.c_str());
      CHECK(s == want);
    };
    { Inst I = base; I.ej[0] = I.ei[0]; expect(I, TNVAN_E_INVALID, "self loop"); }
    { Inst I = base; std::swap(I.ei[1], I.ej[1]); expect(I, TNVAN_E_INVALID, "i > j"); }
    { Inst I = base; I.ei.push_back(I.ei[2]); I.ej.push_back(I.ej[2]); I.J.push_back(1.0);
      expect(I, TNVAN_E_INVALID, "duplicate edge"); }
    { Inst I = base; I.ej[3] = 99; expect(I, TNVAN_E_INVALID, "endpoint out of range"); }
    { Inst I = base; I.J[4] = NAN; expect(I, TNVAN_E_INVALID, "NaN coupling"); }
    { Inst I = base; I.h[2] = INFINITY; expect(I, TNVAN_E_INVALID, "infinite field"); }
    { Inst I = base; I.beta = -1.0; expect(I, TNVAN_E_INVALID, "negative beta"); }
    { Inst I = base; I.order[0] = I.W[0]; expect(I, TNVAN_E_INVALID, "order meets W"); }
    { Inst I = base; I.order.pop_back(); I.gp.back() -= 1; expect(I, TNVAN_E_INVALID, "not covering"); }
    { Inst I = base; I.W.push_back(I.W[0]); I.order.pop_back(); I.gp.back() -= 1;
      expect(I, TNVAN_E_INVALID, "repeated W"); }
    { Inst I = base; I.gp = {0, 12}; expect(I, TNVAN_E_INVALID, "group of 12"); }
    { Inst I = base; I.gp = {0, 3, 2, 12}; expect(I, TNVAN_E_INVALID, "descending groups"); }
    { Inst I = base; I.hidden = -3; expect(I, TNVAN_E_INVALID, "negative hidden width"); }
    { Inst I = lattice(16, {}, true, rng); expect(I, TNVAN_E_INVALID, "row groups of 16"); }
    { Inst I = lattice(16, {}, false, rng); expect(I, TNVAN_E_WIDTH, "strip of 16 columns"); }
  }
  // --- seeded random instances: compile or refuse, nothing else
  int ok = 0, refused = 0;
  for (int it = 0; it < 300; ++it) {
    const int n = 4 + (int)(rng() % 40), d = 2 + (int)(rng() % 4), m = (int)(rng() % (n / 2 + 1));
    Inst I = random_graph(n, d, m, rng);
    if (rng() % 5 == 0) {
      // random groups over the order, sometimes too large
      I.gp = {0};
      while (I.gp.back() < (int)I.order.size())
        I.gp.push_back(std::min<int>((int)I.order.size(), I.gp.back() + 1 + (int)(rng() % 10)));
    }
    if (rng() % 7 == 0 && !I.ei.empty()) I.ei[rng() % I.ei.size()] = -(int)(rng() % 3);
    HostProgram P;
    const tnvan_status s = compile(I, 1 + (int)(rng() % 14), P, msg);
    CHECK(s == TNVAN_OK || s == TNVAN_E_INVALID || s == TNVAN_E_WIDTH);
    (s == TNVAN_OK ? ok : refused) += 1;
  }
  CHECK(ok > 50 && refused > 20);
  // --- planner: the bound holds, W and R partition the vertices
  for (int it = 0; it < 40; ++it) {
    const int n = 20 + (int)(rng() % 200);
    Inst I = random_graph(n, 3 + (int)(rng() % 3), 0, rng);
    const int wu = 1 + (int)(rng() % 8);
    std::vector<int32_t> key;
    if (it % 2) {
      key.resize(n);
      for (int i = 0; i < n; ++i) key[i] = i;
      std::shuffle(key.begin(), key.end(), rng);
    }
    PlanResult R;
    const tnvan_status s = plan_width_set(n, I.ei, I.ej, wu, key, it % 3 == 0, R, msg);
    CHECK(s == TNVAN_OK);
    CHECK(R.width <= wu);
    CHECK((int)(R.W.size() + R.order.size()) == n && (int)R.pi.size() == n);
    std::vector<int> seen(n, 0);
    for (int v : R.W) seen[v] += 1;
    for (int v : R.order) seen[v] += 1;
    for (int v = 0; v < n; ++v) CHECK(seen[v] == 1);
  }
  {
    PlanResult R;
    std::vector<int32_t> ei = {0, 1}, ej = {1, 5}, badkey = {0, 0, 1};
    CHECK(plan_width_set(3, ei, ej, 2, {}, false, R, msg) == TNVAN_E_INVALID);
    CHECK(plan_width_set(3, {0}, {1}, 0, {}, false, R, msg) == TNVAN_E_INVALID);
    CHECK(plan_width_set(3, {0}, {1}, 2, badkey, false, R, msg) == TNVAN_E_INVALID);
    CHECK(plan_width_set(3, {1}, {1}, 2, {}, false, R, msg) == TNVAN_E_INVALID);
  }
  if (g_fail) std::fprintf(stderr, "%d checks failed\n", g_fail);
  else std::printf("host harness ok (%d compiled, %d refused)\n", ok, refused);
  return g_fail ? 1 : 0;
}
