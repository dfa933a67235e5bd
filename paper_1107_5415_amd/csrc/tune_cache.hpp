// The batched autotuner's choices: remembered per process, keyed by the
// device architecture, the plan flags and the exact list of matrices, and
// saved to or merged from a JSON file so that they survive the process.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "plan.hpp"

namespace lfft {

struct TuneKey {
  std::string arch;         // e.g. "gfx950"
  int d = 0;
  uint32_t flags = 0;
  std::vector<i64> Ms;      // every lattice's matrix, row-major, concatenated
  bool operator<(const TuneKey& o) const;
};

struct TuneVal {
  int tile_lg = 12, order = 0;
  float ms = -1.0f;         // time of the chosen configuration when tuned
};

// architecture name of the current device without feature suffixes
// (throws StatusError{E_HIP} without a device)
std::string device_arch();

bool tune_cache_find(const TuneKey& k, TuneVal* v);
void tune_cache_put(const TuneKey& k, const TuneVal& v);
void tune_cache_clear();
int tune_cache_size();
// write every remembered choice (throws E_ARG, E_IO)
void tune_cache_save(const char* path);
// merge the entries of `arch` from a file written by tune_cache_save; the
// whole file is validated first and nothing is taken from a malformed one
// (throws E_ARG, E_IO); returns the number of entries taken
int tune_cache_load(const char* path, const std::string& arch);

}  // namespace lfft
