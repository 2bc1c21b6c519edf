// Host harness for the library's bit-exact scalar arithmetic
// (paper_2603_26968_amd/csrc/lopc_numeric.h, compiled here for the CPU).
// stdin: lines "<y bits hex> <inv bits hex>"; stdout: q_bin and q_bin32 per line.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../paper_2603_26968_amd/csrc/lopc_numeric.h"

int main() {
  unsigned long long yb, ib;
  while (std::scanf("%llx %llx", &yb, &ib) == 2) {
    double y, inv;
    std::memcpy(&y, &yb, 8);
    std::memcpy(&inv, &ib, 8);
    std::printf("%lld %lld\n", (long long)lopc::q_bin(y, inv),
                (long long)lopc::q_bin32(y, inv));
  }
  return 0;
}
