// Host-only check of the tile-scratch invariant of mrv_tiles.hpp, compiled with
// g++ by tests/test_tile_bins.py.  A call plans a chunk floor f (the smallest
// planned tile length of its teams) and dynamic LDS big enough for every team's
// planned chunk; the scratch holds tile_bins(max_T, f) bins.  Whatever chunk a
// team holds when the kernel runs (tilings may change after planning), the chunk
// k_query_info takes must fit the LDS and give at most tile_bins - 2 tiles.
#include <cstdio>
#include <cstdlib>
#include <initializer_list>

#include "mrv_tiles.hpp"

int main()
{
    const int kMaxChunk = 64;
    const long long kMaxT = 1 << 20;
    const int lds_per_t[] = { 16, 1000, 2048, 5440, 9216, 20000, 40000 };
    const long long horizons[] = { 1, 2, 3, 63, 64, 65, 187, 1000, 4095, 4096, 65536, kMaxT - 1, kMaxT };
    long long checks = 0;
    for (int L : lds_per_t)
        for (int floor_c = 1; floor_c <= kMaxChunk; ++floor_c)
            for (int planned = floor_c; planned <= kMaxChunk; planned += 3)
                for (int extra : { 0, 1, 777, 4096 }) {
                    const int lds = planned * L + 64 + extra;
                    if (lds > 160 * 1024) continue;
                    for (int live = 1; live <= kMaxChunk; ++live)
                        for (long long maxT : horizons) {
                            const long long bins = mrv::tile_bins(maxT, floor_c);
                            const int c = mrv::query_chunk(live, lds, L, floor_c, kMaxChunk);
                            ++checks;
                            if (c < floor_c || c < 1 || c > kMaxChunk || (long long)c * L + 64 > lds) {
                                std::printf("bad chunk %d: live %d floor %d L %d lds %d\n", c, live, floor_c, L, lds);
                                return 1;
                            }
                            for (long long T : { maxT, maxT - 1, (maxT + 1) / 2, 1LL }) {
                                if (T < 1) continue;
                                if (mrv::tiles_of(T, c) > bins - 2) {
                                    std::printf("tiles %lld > bins - 2 = %lld: T %lld chunk %d floor %d\n",
                                                mrv::tiles_of(T, c), bins - 2, T, c, floor_c);
                                    return 1;
                                }
                            }
                        }
                }
    std::printf("ok %lld\n", checks);
    return 0;
}
