// Host-side check of the vertex permutation the library uses (device.h):
// perm_apply is a bijection on [0, n) and perm_invert undoes it.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <vector>

#include "device.h"

using namespace hipscc;

int main() {
    for (uint32_t n : {1u, 2u, 3u, 17u, 1000u, 65536u, 65537u, 1000003u}) {
        Perm P;
        P.n = n;
        uint32_t bits = 1;
        while ((1ull << (2 * bits)) < (uint64_t)n) bits++;
        P.half_bits = bits;
        P.key = 0x9E3779B97F4A7C15ull * n + 12345;
        std::vector<char> seen(n, 0);
        for (uint32_t x = 0; x < n; x++) {
            const uint32_t y = perm_apply(P, x);
            if (y >= n || seen[y]) {
                std::printf("not a bijection: n=%u x=%u\n", n, x);
                return 1;
            }
            seen[y] = 1;
            if (perm_invert(P, y) != x) {
                std::printf("inverse fails: n=%u x=%u\n", n, x);
                return 1;
            }
        }
    }
    std::printf("ok\n");
    return 0;
}
