// Autotuner cache file of the batched plan (host code): one entry per line,
// "<key> <cells per lane>", appended after each tuning.
#pragma once

#include <string>

namespace adk {

// The cells-per-lane choice (1, 2 or 4) stored last for key in the file at
// path, 0 when path is null, the file cannot be read or holds no valid entry
// for key.  Lines that do not parse are skipped.
int tune_cache_lookup(const char *path, const std::string &key);

// Appends "<key> <cpl>" to the file at path (nothing when path is null or the
// file cannot be opened).
void tune_cache_store(const char *path, const std::string &key, int cpl);

}  // namespace adk
