// Launch-shape autotuner.  The first time a kernel runs with a given shape
// key, every candidate launch configuration is timed with HIP events on the
// stream the kernel runs on, and the fastest is kept for the rest of the
// process.  With the environment variable WMG_TUNE_CACHE naming a file, the
// choices are read from it at the first lookup and every new choice is
// appended, so later processes skip the search.  WMG_TUNE=0 switches the
// search off (candidate 0, the hand-picked default, everywhere);
// WMG_TUNE_VERBOSE=1 prints every candidate's time to stderr.
//
// Candidates must be pure launches (outputs overwritten from inputs that the
// launch does not modify): tune_choice always ends with one launch of the
// chosen candidate, so its outputs are the chosen candidate's.  No search
// runs while the stream is being captured into a graph.
#include <cstdio>
#include <functional>
#include <cstdlib>
#include <mutex>
#include <string>
#include <unordered_map>

#include "wmg_internal.h"

namespace wmg {

namespace {
struct Entry {
  int choice;
  double ms;
};
std::mutex g_mu;
std::unordered_map<std::string, Entry> g_table;
bool g_loaded = false;
int g_enabled = -1;
bool g_verbose = false;
int g_force = -1;  // test hook: run this candidate everywhere, no search

void load_cache_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char *e = std::getenv("WMG_TUNE");
  g_enabled = !(e && e[0] == '0');
  const char *v = std::getenv("WMG_TUNE_VERBOSE");
  g_verbose = v && v[0] == '1';
  const char *path = std::getenv("WMG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char key[512];
  int choice;
  double ms;
  while (std::fscanf(f, "%511s %d %lf", key, &choice, &ms) == 3) g_table[key] = {choice, ms};
  std::fclose(f);
}

void append_cache_locked(const std::string &key, const Entry &e) {
  const char *path = std::getenv("WMG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %.6f\n", key.c_str(), e.choice, e.ms);
  std::fclose(f);
}
}  // namespace

int tune_choice(const std::string &key, int ncand, const std::function<int(int)> &run, hipStream_t st, int *choice) {
  int known = -1, forced = -1;
  bool search = true;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    if (g_force >= 0) forced = g_force < ncand ? g_force : 0;
    auto it = g_table.find(key);
    if (it != g_table.end() && it->second.choice < ncand) known = it->second.choice;
    search = known < 0 && g_enabled && ncand > 1;
  }
  if (forced >= 0) {
    *choice = forced;
    return run(forced);
  }
  if (search) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    WMG_HIP(hipStreamIsCapturing(st, &cs));
    search = cs == hipStreamCaptureStatusNone;
  }
  if (!search) {
    *choice = known < 0 ? 0 : known;
    return run(*choice);
  }
  hipEvent_t e0, e1;
  WMG_HIP(hipEventCreate(&e0));
  WMG_HIP(hipEventCreate(&e1));
  int best = 0;
  double best_ms = 1e300;
  int rc = 0;
  for (int c = 0; c < ncand && !rc; c++) {
    rc = run(c);  // warm-up (and validity: a candidate that cannot launch is an error)
    if (rc) break;
    if (hipEventRecord(e0, st) != hipSuccess) { rc = set_error(-3, "tune: event record"); break; }
    const int reps = 3;
    for (int k = 0; k < reps && !rc; k++) rc = run(c);
    if (rc) break;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = set_error(-3, "tune: event sync");
      break;
    }
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = set_error(-3, "tune: elapsed time"); break; }
    if (g_verbose) std::fprintf(stderr, "tune %s candidate %d: %.4f ms\n", key.c_str(), c, ms / reps);
    if (ms / reps < best_ms) {
      best_ms = ms / reps;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  // leave the chosen candidate's result in the outputs
  if (best != ncand - 1) {
    rc = run(best);
    if (rc) return rc;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  Entry e{best, best_ms};
  g_table[key] = e;
  append_cache_locked(key, e);
  *choice = best;
  return 0;
}

int tune_lookup(const std::string &key) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache_locked();
  auto it = g_table.find(key);
  return it == g_table.end() ? -1 : it->second.choice;
}

}  // namespace wmg

extern "C" int wmg_tune_force(int choice) {
  std::lock_guard<std::mutex> lk(wmg::g_mu);
  const int prev = wmg::g_force;
  wmg::g_force = choice < 0 ? -1 : choice;
  return prev;
}
