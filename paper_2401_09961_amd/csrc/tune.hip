// Autotuner of the launch shapes: the stencil's band height (blocks of
// rows per workgroup), the block count of the CG update and, for 16-bit MFMA
// products, the product tile (256 x 256 or 128 x 128).  Each candidate is
// timed with HIP events on the caller's stream on the plan's own workspace;
// the fastest is applied.  Choices persist in a JSON file keyed by the
// image shape, the precision, the preconditioner form and the GPU
// architecture, so a shape is measured once per machine.
//
// File format (one entry per line inside "entries", written whole by this
// code and read back line by line):
//   {"irlsu_tune_cache": 1, "entries": [
//   {"kind": "plan", "arch": "gfx950:sramecc+:xnack-", "N": 8192, "M": 8192,
//    "precision": 3, "form": 3, "stencil_rows": 64, "update_blocks": 256,
//    "small_tiles": 0, "stencil_us": 201.3, "update_us": 0, "precond_us": 0},
//   ...
//   ]}
#include "tune.hpp"

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace irlsu {

namespace {

bool parse_line(const char* line, TuneEntry& e) {
  char kind[32] = {0}, arch[128] = {0};
  long long N = 0, M = 0;
  int prec = 0, form = 0, rows = 0, upd = 0, small = 0;
  double su = 0, uu = 0, pu = 0;
  const int n = std::sscanf(
      line,
      " {\"kind\": \"%31[^\"]\", \"arch\": \"%127[^\"]\", \"N\": %lld, \"M\": %lld, "
      "\"precision\": %d, \"form\": %d, \"stencil_rows\": %d, \"update_blocks\": %d, "
      "\"small_tiles\": %d, \"stencil_us\": %lf, \"update_us\": %lf, \"precond_us\": %lf",
      kind, arch, &N, &M, &prec, &form, &rows, &upd, &small, &su, &uu, &pu);
  if (n != 12) return false;
  e.kind = kind;
  e.arch = arch;
  e.N = N;
  e.M = M;
  e.precision = prec;
  e.form = form;
  e.stencil_rows = rows;
  e.update_blocks = upd;
  e.small_tiles = small;
  e.stencil_us = su;
  e.update_us = uu;
  e.precond_us = pu;
  return true;
}

}  // namespace

std::vector<TuneEntry> tune_cache_read(const char* path) {
  std::vector<TuneEntry> out;
  if (!path) return out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  char line[1024];
  while (std::fgets(line, sizeof(line), f)) {
    TuneEntry e;
    if (parse_line(line, e)) out.push_back(e);
  }
  std::fclose(f);
  return out;
}

bool tune_cache_write(const char* path, const std::vector<TuneEntry>& entries) {
  if (!path) return false;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\"irlsu_tune_cache\": 1, \"entries\": [\n");
  for (size_t i = 0; i < entries.size(); ++i) {
    const TuneEntry& e = entries[i];
    std::fprintf(f,
                 "{\"kind\": \"%s\", \"arch\": \"%s\", \"N\": %lld, \"M\": %lld, "
                 "\"precision\": %d, \"form\": %d, \"stencil_rows\": %d, \"update_blocks\": %d, "
                 "\"small_tiles\": %d, \"stencil_us\": %.3f, \"update_us\": %.3f, "
                 "\"precond_us\": %.3f}%s\n",
                 e.kind.c_str(), e.arch.c_str(), (long long)e.N, (long long)e.M, e.precision,
                 e.form, e.stencil_rows, e.update_blocks, e.small_tiles, e.stencil_us,
                 e.update_us, e.precond_us, i + 1 < entries.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

const TuneEntry* tune_cache_find(const std::vector<TuneEntry>& entries, const TuneEntry& key) {
  for (const TuneEntry& e : entries)
    if (e.kind == key.kind && e.arch == key.arch && e.N == key.N && e.M == key.M &&
        e.precision == key.precision && e.form == key.form)
      return &e;
  return nullptr;
}

void tune_cache_put(std::vector<TuneEntry>& entries, const TuneEntry& e) {
  for (TuneEntry& x : entries)
    if (x.kind == e.kind && x.arch == e.arch && x.N == e.N && x.M == e.M &&
        x.precision == e.precision && x.form == e.form) {
      x = e;
      return;
    }
  entries.push_back(e);
}

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  return std::string(prop.gcnArchName);
}

// Mean microseconds per call of `launch` over reps calls after two warm-ups,
// HIP events on stream s; negative on a HIP error.
double time_launches(const std::function<void()>& launch, int reps, hipStream_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  launch();
  launch();
  double us = -1.0;
  if (hipEventRecord(e0, s) == hipSuccess) {
    for (int r = 0; r < reps; ++r) launch();
    float ms = 0.f;
    if (hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
        hipEventElapsedTime(&ms, e0, e1) == hipSuccess && hipGetLastError() == hipSuccess)
      us = 1e3 * (double)ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return us;
}

}  // namespace irlsu
