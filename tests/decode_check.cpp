// Host build of the engine's index decode (decode.h), for the CPU tests.
// Reads commands from stdin:
//   d q x              print QDiv(q).div(x)
//   g q idx r s0 ...   print group_off(idx, {s0 .. s_{r-1}}, r, QDiv(q))
//   s q lo hi          print how many x in [lo, hi) have QDiv(q).div(x) != x / q
#include <cstdint>
#include <cstdio>
#include <vector>

#include "decode.h"

int main() {
  char kind;
  while (std::scanf(" %c", &kind) == 1) {
    int q;
    long long x;
    if (std::scanf("%d %lld", &q, &x) != 2) return 2;
    const kn::QDiv D(q);
    if (kind == 'd') {
      std::printf("%d\n", D.div((int32_t)x));
    } else if (kind == 'g') {
      int r;
      if (std::scanf("%d", &r) != 1) return 2;
      std::vector<int32_t> str(r);
      for (int j = 0; j < r; ++j)
        if (std::scanf("%d", &str[j]) != 1) return 2;
      std::printf("%d\n", kn::group_off((int32_t)x, str.data(), r, D));
    } else if (kind == 's') {
      long long hi;
      if (std::scanf("%lld", &hi) != 1) return 2;
      long long bad = 0;
      for (long long v = x; v < hi; ++v)
        if (D.div((int32_t)v) != (int32_t)(v / q)) ++bad;
      std::printf("%lld\n", bad);
    } else {
      return 2;
    }
  }
  return 0;
}
