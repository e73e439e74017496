// Autotuner of the launch shapes (tnvan_autotune): times the net's own
// calls on the caller's batch for every candidate shape of the kernels the
// net runs and keeps the fastest, with an optional JSON cache keyed by the
// GPU architecture and the net's signature.  A client of the C ABI only
// (tnvan_get_tuning / tnvan_set_tuning and the logZ entry points), plus the
// signature the library reports.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/tnvan.h"
#include "launch.h"

namespace {

using Shapes = std::map<std::string, int>;

// ---------------------------------------------------------------- cache
// {"<key>": {"general_tile_fwd": 4, "general_tile_bwd": 8, "chain_groups": 2}, ...}
struct Reader {
  const std::string &s;
  size_t i = 0;
  void ws() { while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i; }
  bool ch(char c) { ws(); if (i < s.size() && s[i] == c) { ++i; return true; } return false; }
  bool str(std::string &out) {
    ws();
    if (i >= s.size() || s[i] != '"') return false;
    out.clear();
    for (++i; i < s.size() && s[i] != '"'; ++i) {
      if (s[i] == '\\' && i + 1 < s.size()) ++i;
      out += s[i];
    }
    return i < s.size() && s[i++] == '"';
  }
  bool num(long long &v) {
    ws();
    size_t j = i;
    if (j < s.size() && (s[j] == '-' || s[j] == '+')) ++j;
    while (j < s.size() && s[j] >= '0' && s[j] <= '9') ++j;
    if (j == i) return false;
    v = std::stoll(s.substr(i, j - i));
    i = j;
    return true;
  }
};

bool parse_cache(const std::string &text, std::map<std::string, Shapes> &out) {
  Reader r{text};
  if (!r.ch('{')) return false;
  if (r.ch('}')) return true;
  do {
    std::string key;
    if (!r.str(key) || !r.ch(':') || !r.ch('{')) return false;
    Shapes sh;
    if (!r.ch('}')) {
      do {
        std::string f;
        long long v;
        if (!r.str(f) || !r.ch(':') || !r.num(v)) return false;
        sh[f] = (int)v;
      } while (r.ch(','));
      if (!r.ch('}')) return false;
    }
    out[key] = sh;
  } while (r.ch(','));
  return r.ch('}');
}

void read_cache(const char *path, std::map<std::string, Shapes> &out) {
  FILE *f = std::fopen(path, "rb");
  if (!f) return;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
  std::fclose(f);
  std::map<std::string, Shapes> m;
  if (parse_cache(text, m)) out.swap(m);   // an unreadable file is replaced
}

bool write_cache(const char *path, const std::map<std::string, Shapes> &m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  std::fprintf(f, "{");
  bool first = true;
  for (auto &e : m) {
    std::fprintf(f, "%s\n  \"%s\": {", first ? "" : ",", e.first.c_str());
    bool f2 = true;
    for (auto &kv : e.second) {
      std::fprintf(f, "%s\"%s\": %d", f2 ? "" : ", ", kv.first.c_str(), kv.second);
      f2 = false;
    }
    std::fprintf(f, "}");
    first = false;
  }
  std::fprintf(f, "\n}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

Shapes to_shapes(const tnvan_tuning &t) {
  return {{"general_tile_fwd", t.general_tile_fwd},
          {"general_tile_bwd", t.general_tile_bwd},
          {"chain_groups", t.chain_groups},
          {"checkpoint_every", t.checkpoint_every},
          {"launch_mode", t.launch_mode}};
}

void from_shapes(const Shapes &s, tnvan_tuning &t) {
  auto get = [&](const char *k) { auto it = s.find(k); return it == s.end() ? 0 : it->second; };
  t.general_tile_fwd = get("general_tile_fwd");
  t.general_tile_bwd = get("general_tile_bwd");
  t.chain_groups = get("chain_groups");
  t.checkpoint_every = get("checkpoint_every");
  t.launch_mode = get("launch_mode");
}

}  // namespace

extern "C" tnvan_status tnvan_autotune(tnvan_net *net, const int64_t *n_samples,
                                       const int8_t *spins, const double *grad_logz,
                                       double *logz, double *dh, double *dJ, double *dbeta,
                                       const char *cache_path, tnvan_tuning *out,
                                       void *stream) {
  if (!net || !n_samples || !out) {
    tnvan::set_last_error("net, n_samples and out are required");
    return TNVAN_E_INVALID;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  tnvan_tuning cur{};
  if (tnvan_status s = tnvan_get_tuning(net, &cur)) return s;
  // the key: architecture, the net's signature, batch size bucket
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    tnvan::set_last_error("hipGetDeviceProperties failed");
    return TNVAN_E_HIP;
  }
  int64_t total = 0;
  std::string sig;
  if (tnvan_status s = tnvan::net_signature(net, sig)) return s;
  std::vector<int64_t> counts;
  for (int q = 0; q < tnvan::net_instances(net); ++q) {
    total += n_samples[q];
    counts.push_back(n_samples[q]);
  }
  int bucket = 0;
  while (((int64_t)1 << bucket) < total) ++bucket;
  const std::string key = std::string(prop.gcnArchName) + "|" + sig + "|B" + std::to_string(bucket);
  std::map<std::string, Shapes> cache;
  if (cache_path) {
    read_cache(cache_path, cache);
    auto it = cache.find(key);
    if (it != cache.end()) {
      tnvan_tuning t{};
      from_shapes(it->second, t);
      t.arena_limit_mib = cur.arena_limit_mib;
      if (tnvan_set_tuning(net, &t) == TNVAN_OK) return tnvan_get_tuning(net, out);
    }
  }
  // time one candidate: a call that lays the tables out, then reps calls
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    tnvan::set_last_error("hipEventCreate failed");
    return TNVAN_E_HIP;
  }
  auto timed = [&](bool bwd, double &ms) -> tnvan_status {
    auto call = [&]() {
      return bwd ? tnvan_logz_backward(net, counts.data(), spins, grad_logz, dh, dJ, dbeta, stream)
                 : tnvan_logz_batch(net, counts.data(), spins, logz, nullptr, stream);
    };
    if (tnvan_status s = call()) return s;
    const int reps = 5;
    if (hipEventRecord(e0, st) != hipSuccess) return TNVAN_E_HIP;
    for (int r = 0; r < reps; ++r)
      if (tnvan_status s = call()) return s;
    float t = 0.f;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess)
      return TNVAN_E_HIP;
    ms = t / reps;
    return TNVAN_OK;
  };
  tnvan_tuning best{};
  best.general_tile_fwd = best.general_tile_bwd = best.chain_groups = best.checkpoint_every = 0;
  best.launch_mode = 0;
  best.arena_limit_mib = cur.arena_limit_mib;
  tnvan_status status = TNVAN_OK;
  // coordinate by coordinate: each field over its candidates with the others
  // at their best so far; the default rule (0) stays unless another
  // candidate is at least 2% faster
  struct Field { int32_t tnvan_tuning::*f; bool bwd; std::vector<int> cand; int kind; };
  const std::vector<Field> fields = {
      {&tnvan_tuning::general_tile_fwd, false, {1, 2, 4, 8, 16, 32, 64}, TNVAN_TUNE_GENERAL},
      {&tnvan_tuning::general_tile_bwd, true, {1, 2, 4, 8, 16, 32, 64}, TNVAN_TUNE_GENERAL},
      {&tnvan_tuning::chain_groups, false, {1, 2}, TNVAN_TUNE_REG_CHAIN},
      {&tnvan_tuning::checkpoint_every, true, {1, 2, 4}, TNVAN_TUNE_REG_CHAIN},
      {&tnvan_tuning::launch_mode, true, {2}, TNVAN_TUNE_GENERAL | TNVAN_TUNE_REG_CHAIN}};
  for (const Field &fd : fields) {
    if (!(cur.kinds & fd.kind)) continue;
    tnvan_tuning t = best;
    t.*(fd.f) = 0;
    double base = 0.0;
    if ((status = tnvan_set_tuning(net, &t)) || (status = timed(fd.bwd, base))) break;
    int pick = 0;
    double pick_ms = base;
    for (int v : fd.cand) {
      t.*(fd.f) = v;
      if (tnvan_set_tuning(net, &t) != TNVAN_OK) continue;   // does not fit
      double ms = 0.0;
      if ((status = timed(fd.bwd, ms))) break;
      if (ms < pick_ms && ms < 0.98 * base) { pick = v; pick_ms = ms; }
    }
    if (status) break;
    best.*(fd.f) = pick;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status) return status;
  if (tnvan_status s = tnvan_set_tuning(net, &best)) return s;
  if (cache_path) {
    cache[key] = to_shapes(best);
    if (!write_cache(cache_path, cache)) {
      tnvan::set_last_error("cannot write the tuning cache");
      return TNVAN_E_INVALID;
    }
  }
  return tnvan_get_tuning(net, out);
}
