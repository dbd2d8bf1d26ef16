// Tuned plan parameters from the autotuner's JSON table (see tuning.cpp).
#pragma once

#include <cstdint>
#include <string>

namespace tacho {

// 0 = not in the table (the option or the library default applies).
struct TunedParams {
  bool found_workload = false, found_order = false;
  int32_t asm_cols = 0, solo_m = 0, solve_level_fronts = 0;  // workload class
  int32_t u_range = 0, chain_min = 0, chain_inplace = 0;     // per precision
};

std::string workload_class_key(int64_t n, int64_t nnz, int precision_fp32);
std::string order_key(int precision_fp32);

// Reads `path`; returns 0, or -1 with `err` set when the file is missing or
// malformed.  Entries absent from the table leave their fields 0.
int load_tuned(const std::string& path, int64_t n, int64_t nnz, int precision_fp32,
               TunedParams& out, std::string& err);

}  // namespace tacho
