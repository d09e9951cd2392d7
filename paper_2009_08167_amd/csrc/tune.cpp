// Measured choice of the sweep decomposition of a problem, with an on-disk
// cache.
//
// The forward/backward elimination (Sec. 4.2, applied once per Lanczos step
// of the shift-and-invert operator) is swept level by level below a cut
// height and through the explicit inverse of the top tree levels above it;
// optionally the bottom heights are swept in one launch per subtree.  The
// cut is chosen at set-up from a cost model of launch latency and bytes.
// Tuning instead times, on the problem itself, one factorisation and a
// sweep pair (out of cache, as in the eigensolver) for every cut within the
// size limits (and none), and keeps the fastest by
//     sweep pair + factorisation / FB_PER_FACT
// if it beats the configuration in place by more than 3%,
// the weight of a factorisation against the sweeps of one shift in the
// eigensolver (about 70 sweep pairs per factorisation on the 2D and 3D
// workloads).  Fused bottom heights are not among the candidates (the
// choice leaves them off): timed alone their sweeps can come out faster by
// a few per cent, while inside the eigensolver, next to the look-ahead
// factorisation and a second spectrum slice on other streams, they made
// the 2D 256^2 p = 3 solve 8-10% slower at every cut.  The choice is stored under a key of the device and of the
// elimination tree; problems set up later with the same key take it.  Every
// candidate is a different order of the same exact operations, so results
// differ between choices only by rounding; a given choice gives the same
// results every time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <unistd.h>
#include <vector>

#include "problem.h"

namespace riga {
namespace {

constexpr double FB_PER_FACT = 70.0;
std::mutex g_tune_mu;

// the cache file: RIGA_TUNE_CACHE, else $XDG_CACHE_HOME/riga/tune.txt,
// else $HOME/.cache/riga/tune.txt ("" when none can be named)
std::string cache_path() {
  if (const char* v = std::getenv("RIGA_TUNE_CACHE")) return v;
  if (const char* v = std::getenv("XDG_CACHE_HOME"); v && *v) return std::string(v) + "/riga/tune.txt";
  if (const char* v = std::getenv("HOME"); v && *v) return std::string(v) + "/.cache/riga/tune.txt";
  return "";
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

// device (architecture, compute units) and elimination tree (fronts'
// orders, fully-summed orders, parents, heights)
std::string tune_key(const riga_problem* pr) {
  hipDeviceProp_t prop{};
  HIPCHECK(hipGetDeviceProperties(&prop, pr->device));
  const Analysis& an = pr->an;
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, an.f_f.data(), an.f_f.size() * sizeof(int32_t));
  h = fnv1a(h, an.f_k.data(), an.f_k.size() * sizeof(int32_t));
  h = fnv1a(h, an.f_parent.data(), an.f_parent.size() * sizeof(int32_t));
  h = fnv1a(h, an.f_height.data(), an.f_height.size() * sizeof(int32_t));
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s/%d/N%lld/F%d/%016llx", arch.c_str(), prop.multiProcessorCount,
                (long long)an.N, an.n_fronts, (unsigned long long)h);
  return buf;
}

struct Entry {
  int cut = -1, fused = 0;
  double sweep_us = 0.0, fact_us = 0.0;
};

std::map<std::string, Entry> read_cache(const std::string& path) {
  std::map<std::string, Entry> m;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream is(line);
    std::string k;
    Entry e;
    if (is >> k >> e.cut >> e.fused >> e.sweep_us >> e.fact_us) m[k] = e;
  }
  return m;
}

void make_dirs(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
}

// replaces (or adds) the key's line; written to a temporary file and
// renamed, so that readers see the old or the new file whole
void write_cache(const std::string& path, const std::string& key, const Entry& e) {
  std::map<std::string, Entry> m = read_cache(path);
  m[key] = e;
  make_dirs(path);
  const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) throw Error(RIGA_EINVAL, "cannot write the tuning cache " + tmp);
    out << "# key top_cut fused_heights sweep_pair_us factorisation_us\n";
    for (const auto& [k, v] : m) {
      char buf[96];
      std::snprintf(buf, sizeof buf, " %d %d %.3f %.3f\n", v.cut, v.fused, v.sweep_us, v.fact_us);
      out << k << buf;
    }
    if (!out) throw Error(RIGA_EINVAL, "cannot write the tuning cache " + tmp);
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    throw Error(RIGA_EINVAL, "cannot replace the tuning cache " + path);
  }
}

void invalidate_factors(riga_problem* pr) {
  for (SolveCtx& c : pr->ctx)
    for (Factor& F : c.fac) {
      F.factored = false;
      F.pre = false;
    }
}

void configure(riga_problem* pr, int cut, int fused) {
  setup_top(pr, cut);
  setup_subtrees(pr, fused);
  HIPCHECK(hipStreamSynchronize(pr->home));
}

}  // namespace

bool tune_lookup(const riga_problem* pr, int* cut, int* fused) {
  const std::string path = cache_path();
  if (path.empty()) return false;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  struct stat sb;
  if (stat(path.c_str(), &sb) != 0) return false;
  const std::map<std::string, Entry> m = read_cache(path);
  const auto it = m.find(tune_key(pr));
  if (it == m.end()) return false;
  *cut = it->second.cut;
  *fused = it->second.fused;
  return true;
}

void tune_problem(riga_problem* pr, int precision, int reps, riga_tune_result* out) {
  hipStream_t s = pr->home;
  const int64_t n = pr->an.N;
  DBuf<double> b, x;
  b.alloc(n, s);
  x.alloc(n, s);
  std::vector<double> hb(n);
  for (int64_t i = 0; i < n; ++i) hb[i] = 1.0 + 1e-3 * (double)(i % 97);
  HIPCHECK(hipMemcpyAsync(b.p, hb.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHECK(hipStreamSynchronize(s));
  // In the eigensolver the Gram-Schmidt passes between two sweeps stream
  // more than the last-level cache holds, so each sweep pair starts with
  // its factor out of the caches: every timed pair here follows a write of
  // FLUSH_BYTES (timed apart from it).
  constexpr size_t FLUSH_BYTES = (size_t)320 << 20;
  DBuf<uint8_t> flush;
  flush.alloc(FLUSH_BYTES, s);
  std::vector<hipEvent_t> evs(2 * (size_t)reps, nullptr);
  struct EventList {
    std::vector<hipEvent_t>& v;
    ~EventList() {
      for (hipEvent_t e : v)
        if (e) (void)hipEventDestroy(e);
    }
  } evl{evs};
  for (hipEvent_t& e : evs) HIPCHECK(hipEventCreate(&e));
  Factor& F = pr->ctx[0].current();
  // one candidate: best of two factorisations (host clock: the call waits
  // for its end) and the median of `reps` sweep pairs, each after a flush
  auto measure = [&](Entry& e) {
    factor_reserve(pr, F, precision, s);
    double fact = 1e300;
    for (int r = 0; r < 2; ++r) {
      const auto t0 = std::chrono::steady_clock::now();
      factor_numeric(pr, F, 0.0, precision, s);
      fact = std::min(fact, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    }
    for (int r = 0; r < 2; ++r) solve_fb(pr, F, b.p, x.p, s);
    for (int q = 0; q < reps; ++q) {
      HIPCHECK(hipMemsetAsync(flush.p, q & 0xff, FLUSH_BYTES, s));
      HIPCHECK(hipEventRecord(evs[2 * q], s));
      solve_fb(pr, F, b.p, x.p, s);
      HIPCHECK(hipEventRecord(evs[2 * q + 1], s));
    }
    HIPCHECK(hipStreamSynchronize(s));
    std::vector<double> t(reps);
    for (int q = 0; q < reps; ++q) {
      float ms = 0.0f;
      HIPCHECK(hipEventElapsedTime(&ms, evs[2 * q], evs[2 * q + 1]));
      t[q] = 1e3 * (double)ms;
    }
    std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
    e.sweep_us = t[reps / 2];
    e.fact_us = 1e6 * fact;
  };
  auto score = [](const Entry& e) { return e.sweep_us + e.fact_us / FB_PER_FACT; };
  // the configuration in place first (the model's, or an earlier choice);
  // another replaces it only when it is faster by more than TUNE_MARGIN, so
  // that differences within the timing noise do not move the choice
  constexpr double TUNE_MARGIN = 0.03;
  Entry before;
  before.cut = pr->top.cut;
  before.fused = pr->sub.nh;
  measure(before);
  Entry best = before;
  int tried = 1;
  for (int cut : top_cut_candidates(pr)) {
    configure(pr, cut, 0);
    Entry e;
    e.cut = pr->top.cut;
    e.fused = pr->sub.nh;
    if (e.cut == before.cut && e.fused == before.fused) continue;
    measure(e);
    ++tried;
    if (score(e) < (1.0 - TUNE_MARGIN) * score(before) && score(e) < score(best)) best = e;
  }
  configure(pr, best.cut, best.fused);
  invalidate_factors(pr);
  const std::string path = cache_path();
  if (!path.empty()) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    write_cache(path, tune_key(pr), best);
  }
  if (out) {
    out->top_cut = best.cut;
    out->fused_heights = best.fused;
    out->candidates = tried;
    out->sweep_us = best.sweep_us;
    out->fact_us = best.fact_us;
    out->before_top_cut = before.cut;
    out->before_fused_heights = before.fused;
    out->before_sweep_us = before.sweep_us;
    out->before_fact_us = before.fact_us;
  }
}

}  // namespace riga
