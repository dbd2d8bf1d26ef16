// Shared host-side definitions of the MI355X supernodal Cholesky library.
#pragma once

#include <cstdint>
#include <string>

namespace tacho {

enum Status : int {
  kOk = 0,
  kInvalid = -1,
  kPattern = -2,
  kNotSpd = -3,
  kNoMemory = -4,
  kHip = -5,
};

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

}  // namespace tacho
