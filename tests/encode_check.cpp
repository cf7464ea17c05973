// Host check of the value dictionary (encode_values in csrc/hier_host.hpp):
// codes decode to the values bit for bit, at most 256 distinct values are
// coded (257 are not), and values that differ only in their bits (signed
// zeros, NaN payloads) keep separate codes.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

#include "hier_host.hpp"

using namespace mvamg;

#define CHECK(c, msg)                                   \
  do {                                                  \
    if (!(c)) {                                         \
      std::fprintf(stderr, "check failed: %s\n", msg); \
      return 1;                                         \
    }                                                   \
  } while (0)

static bool decodes(const std::vector<double>& v, const std::vector<uint8_t>& code, const std::vector<double>& tab) {
  if (code.size() != v.size()) return false;
  for (size_t i = 0; i < v.size(); ++i)
    if (code[i] >= tab.size() || std::memcmp(&tab[code[i]], &v[i], sizeof(double)) != 0) return false;
  return true;
}

int main() {
  std::vector<uint8_t> code;
  std::vector<double> tab;
  // 256 distinct values, repeated and shuffled: coded
  std::vector<double> v;
  for (int r = 0; r < 3; ++r)
    for (int i = 0; i < 256; ++i) v.push_back(std::ldexp(1.0 + i, -7 * (i % 5)) * ((i * 37) % 2 ? -1.0 : 1.0));
  for (size_t i = 0; i < v.size(); ++i) std::swap(v[i], v[(i * 7919) % v.size()]);
  std::vector<double> u(v);
  std::sort(u.begin(), u.end());
  const size_t distinct = (size_t)(std::unique(u.begin(), u.end()) - u.begin());
  CHECK(distinct <= 256, "test input");
  CHECK(encode_values(v, code, tab) && tab.size() == distinct && decodes(v, code, tab), "256 distinct values coded");
  // one more distinct value: not coded, outputs cleared
  std::vector<double> w;
  for (int i = 0; i < 257; ++i) w.push_back(0.5 + i);
  CHECK(!encode_values(w, code, tab) && code.empty() && tab.empty(), "257 distinct values not coded");
  // signed zeros and two NaN payloads are four values
  double nan1 = std::numeric_limits<double>::quiet_NaN(), nan2;
  uint64_t b;
  std::memcpy(&b, &nan1, 8);
  b ^= 1;
  std::memcpy(&nan2, &b, 8);
  std::vector<double> z = {0.0, -0.0, nan1, nan2, 0.0, -0.0};
  CHECK(encode_values(z, code, tab) && tab.size() == 4 && decodes(z, code, tab), "bitwise distinct values");
  CHECK(code[0] != code[1] && code[0] == code[4] && code[1] == code[5] && code[2] != code[3], "codes by bits");
  // empty input: nothing to code
  std::vector<double> e;
  CHECK(!encode_values(e, code, tab), "empty input");
  std::printf("ok\n");
  return 0;
}
