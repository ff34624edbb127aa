// Host-side walk over every single and spin-conserving double of a complete
// pool: each must get its own slot of the generator table, inside the table.
#include "conn_ops.h"
#include <cstdio>
#include <vector>
using namespace swcs;
int main() {
  int bad = 0;
  for (int nsp : {1, 2, 3, 7, 26, 32}) {
    const int nso = 2 * nsp;
    const long long size = optab_size(nsp), npairs = (long long)nso * (nso - 1) / 2;
    std::vector<int> seen((size_t)size, 0);
    long long used = 0;
    for (int P = 0; P < nso; ++P)
      for (int Q = 0; Q < P; ++Q) {
        if ((P & 1) == (Q & 1)) {
          const long long s = pair_index(P, Q);
          if (s < 0 || s >= npairs || seen[s]++) ++bad;
          ++used;
        }
        for (int R = 0; R < nso; ++R)
          for (int S = 0; S < R; ++S) {
            if (R == P || R == Q || S == P || S == Q) continue;
            if ((P & 1) + (Q & 1) != (R & 1) + (S & 1)) continue;
            if (!(P > R || (P == R && Q > S))) continue;
            const long long s = optab_double_slot(nsp, P, Q, R, S);
            if (s < npairs || s >= size || seen[s]++) ++bad;
            ++used;
          }
      }
    printf("nsp %d size %lld used %lld\n", nsp, size, used);
  }
  printf("bad %d\n", bad);
  return bad != 0;
}
