// Autotuner cache (JSON file) and timing helpers; see tune.hip.
#pragma once

#include <functional>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace irlsu {

struct TuneEntry {
  std::string kind;   // "plan" or "batch_tile"
  std::string arch;   // gcnArchName of the device
  int64_t N = 0, M = 0;
  int precision = 0;  // irlsu_precision
  int form = 0;       // IRLSU_PLAN_* of the plan (batch tiles: 0 grouped products, 3 fast)
  int stencil_rows = 0, update_blocks = 0, small_tiles = 0;
  double stencil_us = 0, update_us = 0, precond_us = 0;
};

std::vector<TuneEntry> tune_cache_read(const char* path);
bool tune_cache_write(const char* path, const std::vector<TuneEntry>& entries);
const TuneEntry* tune_cache_find(const std::vector<TuneEntry>& entries, const TuneEntry& key);
void tune_cache_put(std::vector<TuneEntry>& entries, const TuneEntry& e);
std::string device_arch(int device);
double time_launches(const std::function<void()>& launch, int reps, hipStream_t s);

}  // namespace irlsu
