// Autotuner for the mixed-precision product kernels (see tda_internal.h).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "tda_internal.h"

namespace tda {
namespace {

struct Tuner {
  std::mutex mu;
  std::map<std::tuple<std::string, int, int>, int> choice;
  bool loaded = false;

  static int bucket(int64_t x) {
    int b = 0;
    while (((int64_t)1 << b) < x) ++b;
    return b;
  }
  void load() {
    if (loaded) return;
    loaded = true;
    const char *path = getenv("TDA_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char name[64];
    int rb, tb, v;
    while (fscanf(f, "%63s %d %d %d", name, &rb, &tb, &v) == 4) choice[{name, rb, tb}] = v;
    fclose(f);
  }
  void save() {
    const char *path = getenv("TDA_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    for (auto &kv : choice)
      fprintf(f, "%s %d %d %d\n", std::get<0>(kv.first).c_str(), std::get<1>(kv.first),
              std::get<2>(kv.first), kv.second);
    fclose(f);
  }
};

Tuner &tuner() {
  static Tuner t;
  return t;
}

}  // namespace

int autotune_pick(const char *kernel, int64_t rows, int64_t templates, const int *variants,
                  int n_variants, hipStream_t s, hipError_t (*launch)(void *ctx, int variant),
                  void *ctx) {
  Tuner &t = tuner();
  // TDA_PRODUCT_VARIANT=<v> forces variant v of every tuned kernel that has one
  if (const char *force = getenv("TDA_PRODUCT_VARIANT")) {
    const int v = atoi(force);
    for (int k = 0; k < n_variants; ++k)
      if (variants[k] == v) return v;
  }
  const char *env = getenv("TDA_AUTOTUNE");
  if (n_variants <= 1 || (env && env[0] == '0')) return variants[0];
  std::lock_guard<std::mutex> lk(t.mu);
  t.load();
  const auto key = std::make_tuple(std::string(kernel), Tuner::bucket(rows), Tuner::bucket(templates));
  auto it = t.choice.find(key);
  if (it != t.choice.end()) return it->second;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return variants[0];
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return variants[0];
  }
  int best = variants[0];
  float best_ms = 1e30f;
  const char *verbose = getenv("TDA_AUTOTUNE_VERBOSE");
  for (int k = 0; k < n_variants; ++k) {
    // the second of two launches: the first also pays for loading the code object
    float ms = 0.f;
    bool ok = true;
    for (int rep = 0; rep < 2 && ok; ++rep)
      ok = hipEventRecord(a, s) == hipSuccess && launch(ctx, variants[k]) == hipSuccess &&
           hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
           hipEventElapsedTime(&ms, a, b) == hipSuccess;
    if (!ok) continue;
    if (verbose && verbose[0] == '1')
      fprintf(stderr, "[autotune] %s rows=%lld templates=%lld variant %d: %.3f ms\n", kernel,
              (long long)rows, (long long)templates, variants[k], ms);
    if (ms < best_ms) {
      best_ms = ms;
      best = variants[k];
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  t.choice[key] = best;
  t.save();
  return best;
}

}  // namespace tda
