// Tuned plan parameters read from the autotuner's JSON table.
//
// The table maps a key to {"params": {name: integer, ...}, "info": {...}}.
// Two kinds of keys are used:
//   "n~2^<lg>/deg<d>/<fp64|fp32>"  a workload class (order rounded to a power
//        of two, mean row degree rounded to an integer): the parameters that
//        only regroup work into tasks and launches (asm_cols, solo_m,
//        solve_level_fronts), whose results are bitwise the same for every
//        setting;
//   "order/<fp64|fp32>"  one entry per precision: the parameters that change
//        the order in which a front's contributions are summed (u_range,
//        chain_min, chain_inplace).  Keeping them independent of the
//        workload keeps a system's result independent of the batch it is
//        factored in, and of the size of the problem around it.
// Only the fields needed here are interpreted; the rest of the file is
// parsed and skipped.
#include <cctype>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "tuning.hpp"

namespace tacho {
namespace {

struct Parser {
  const std::string& s;
  size_t i = 0;
  std::string err;

  explicit Parser(const std::string& text) : s(text) {}

  void ws() {
    while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool fail(const std::string& m) {
    if (err.empty()) err = m + " at offset " + std::to_string(i);
    return false;
  }
  bool string(std::string& out) {
    ws();
    if (i >= s.size() || s[i] != '"') return fail("expected a string");
    ++i;
    out.clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\') {
        if (i + 1 >= s.size()) return fail("bad escape");
        const char e = s[i + 1];
        out.push_back(e == 'n' ? '\n' : e == 't' ? '\t' : e);
        i += 2;
        if (e == 'u') i += 4;  // \uXXXX: not needed by any key, skipped
      } else {
        out.push_back(s[i++]);
      }
    }
    if (i >= s.size()) return fail("unterminated string");
    ++i;
    return true;
  }
  bool number(double& out) {
    ws();
    const char* b = s.c_str() + i;
    char* e = nullptr;
    out = std::strtod(b, &e);
    if (e == b) return fail("expected a number");
    i += (size_t)(e - b);
    return true;
  }
  // Skip any value.
  bool skip() {
    ws();
    if (i >= s.size()) return fail("unexpected end");
    const char c = s[i];
    if (c == '{') {
      ++i;
      if (eat('}')) return true;
      do {
        std::string k;
        if (!string(k) || !eat(':') || !skip()) return fail("bad object");
      } while (eat(','));
      return eat('}') || fail("expected '}'");
    }
    if (c == '[') {
      ++i;
      if (eat(']')) return true;
      do {
        if (!skip()) return false;
      } while (eat(','));
      return eat(']') || fail("expected ']'");
    }
    if (c == '"') {
      std::string t;
      return string(t);
    }
    for (const char* lit : {"true", "false", "null"})
      if (s.compare(i, std::strlen(lit), lit) == 0) {
        i += std::strlen(lit);
        return true;
      }
    double d;
    return number(d);
  }
  // {"name": integer, ...}
  bool params(std::map<std::string, int64_t>& out) {
    if (!eat('{')) return fail("expected '{'");
    if (eat('}')) return true;
    do {
      std::string k;
      double v;
      if (!string(k) || !eat(':') || !number(v)) return fail("bad parameter");
      if (v != (double)(int64_t)v) return fail("parameter " + k + " is not an integer");
      out[k] = (int64_t)v;
    } while (eat(','));
    return eat('}') || fail("expected '}'");
  }
  // {key: {"params": {...}, "info": {...}}, ...}
  bool table(std::map<std::string, std::map<std::string, int64_t>>& out) {
    if (!eat('{')) return fail("expected '{'");
    if (eat('}')) return true;
    do {
      std::string key;
      if (!string(key) || !eat(':') || !eat('{')) return fail("bad entry");
      auto& dst = out[key];
      if (!eat('}')) {
        do {
          std::string field;
          if (!string(field) || !eat(':')) return fail("bad entry field");
          if (field == "params") {
            if (!params(dst)) return false;
          } else if (!skip()) {
            return false;
          }
        } while (eat(','));
        if (!eat('}')) return fail("expected '}'");
      }
    } while (eat(','));
    if (!eat('}')) return fail("expected '}'");
    ws();
    return i == s.size() || fail("trailing characters");
  }
};

}  // namespace

std::string workload_class_key(int64_t n, int64_t nnz, int precision_fp32) {
  // lg: the integer closest to log2(n) (2^lg <= n < 2^(lg+1), rounded up when
  // n^2 >= 2^(2 lg + 1)); deg: nnz / n rounded half up.  Exact integer rules,
  // shared with the Python table writer.
  const int64_t nn = n > 1 ? n : 1;
  int lg = 0;
  while ((nn >> (lg + 1)) > 0) ++lg;
  if ((unsigned __int128)nn * (unsigned __int128)nn >= ((unsigned __int128)1 << (2 * lg + 1))) ++lg;
  const int64_t deg = (2 * nnz + nn) / (2 * nn);
  return "n~2^" + std::to_string(lg) + "/deg" + std::to_string(deg) + "/" +
         (precision_fp32 ? "fp32" : "fp64");
}

std::string order_key(int precision_fp32) {
  return std::string("order/") + (precision_fp32 ? "fp32" : "fp64");
}

int load_tuned(const std::string& path, int64_t n, int64_t nnz, int precision_fp32,
               TunedParams& out, std::string& err) {
  std::ifstream in(path, std::ios::binary);
  if (!in) {
    err = "cannot read the tuning table " + path;
    return -1;
  }
  std::stringstream ss;
  ss << in.rdbuf();
  const std::string text = ss.str();
  Parser p(text);
  std::map<std::string, std::map<std::string, int64_t>> tab;
  if (!p.table(tab)) {
    err = "tuning table " + path + ": " + p.err;
    return -1;
  }
  out = TunedParams();
  auto take = [&](const std::map<std::string, int64_t>& e, const char* name, int32_t& dst) {
    auto it = e.find(name);
    if (it != e.end()) dst = (int32_t)it->second;
  };
  auto w = tab.find(workload_class_key(n, nnz, precision_fp32));
  if (w != tab.end()) {
    out.found_workload = true;
    take(w->second, "asm_cols", out.asm_cols);
    take(w->second, "solo_m", out.solo_m);
    take(w->second, "solve_level_fronts", out.solve_level_fronts);
  }
  auto o = tab.find(order_key(precision_fp32));
  if (o != tab.end()) {
    out.found_order = true;
    take(o->second, "u_range", out.u_range);
    take(o->second, "chain_min", out.chain_min);
    take(o->second, "chain_inplace", out.chain_inplace);
  }
  return 0;
}

}  // namespace tacho
