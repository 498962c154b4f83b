// Host-only check of the rollout tile's LDS fitting rule (mppi_internal.hpp):
// reads "J T n S sgf_m" lines and prints "fits chunk_steps lds_bytes
// keeps_noise" for each, so the Python test can check the rule's invariants.
#include <cstdio>

#include "mppi_internal.hpp"

int main()
{
    int J, T, n, S, m;
    while (std::scanf("%d %d %d %d %d", &J, &T, &n, &S, &m) == 5) {
        const int tc = dbas::tile_chunk_steps(J, T, n, S);
        const bool fits = dbas::tile_fits(J, T, n, S, m);
        const size_t lds = tc > 0 ? dbas::tile_lds_bytes(J, T, n, S) : 0;
        std::printf("%d %d %zu %d\n", fits ? 1 : 0, tc, lds, dbas::tile_keeps_noise(J, T, n, S) ? 1 : 0);
    }
    return 0;
}
