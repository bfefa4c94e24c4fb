// Drives the server's range allocator from a script on stdin (test harness, host only).
//   C capacity align   reset        A bytes   alloc -> prints offset or -1
//   R offset bytes     release      S         prints used, free ranges, largest
#include <cstdio>
#include <cstring>
#include "arena.h"

int main() {
  tmfg::RangeAllocator a;
  char op[4];
  while (std::scanf("%3s", op) == 1) {
    if (!std::strcmp(op, "C")) {
      unsigned long long c, al;
      std::scanf("%llu %llu", &c, &al);
      a.reset(c, al);
    } else if (!std::strcmp(op, "A")) {
      unsigned long long b;
      std::scanf("%llu", &b);
      size_t off;
      if (a.alloc(b, &off)) std::printf("%llu\n", (unsigned long long)off);
      else std::printf("-1\n");
    } else if (!std::strcmp(op, "R")) {
      unsigned long long o, b;
      std::scanf("%llu %llu", &o, &b);
      a.release(o, b);
    } else if (!std::strcmp(op, "S")) {
      std::printf("%llu %llu %llu\n", (unsigned long long)a.used(), (unsigned long long)a.ranges(),
                  (unsigned long long)a.largest());
    }
  }
  return 0;
}
