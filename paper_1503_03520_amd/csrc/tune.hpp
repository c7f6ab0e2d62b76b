// The library's autotuner cache: the launch choices it measured, by key
// (e.g. "fista_f32_residual/27": the residual-pass variant for rows in
// (2^26, 2^27]).  Lookups and stores are thread-safe.  With L1LS_TUNE_CACHE
// set to a file path the cache is read from that JSON file on first use and
// written back after every new choice, so later processes skip the timing.
#pragma once

#include <cstdint>
#include <string>

int tune_lookup(const std::string& key);          // -1: not measured yet
void tune_store(const std::string& key, int choice);
int tune_size_class(int64_t rows);                // ceil(log2(rows))
