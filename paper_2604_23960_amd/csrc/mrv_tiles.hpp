// Tile arithmetic shared by the host runtime (scratch sizing) and the device
// (k_query_info).  Plain C++ with no HIP dependency, so a host-only test can
// compile it on its own and check the invariant stated below.
//
// A call's tile-enumeration scratch holds tile_bins(max_T, chunk_floor) bins,
// where max_T bounds every query's horizon and chunk_floor is the smallest
// tile length the call was planned with.  query_chunk() never returns less
// than chunk_floor, whatever the team's current setting, so a query's tile
// count tiles_of(T, chunk) never exceeds tile_bins(max_T, chunk_floor) - 2 (the
// largest bin index the kernels write is the tile count itself).
#pragma once

#if defined(__HIP__)
#define MRV_HD __attribute__((host, device))
#else
#define MRV_HD
#endif

namespace mrv {

// Timesteps per tile of one query: the team's current setting, no more than
// the launch's dynamic LDS holds (64 bytes of it are reserved), no fewer than
// the floor the call's scratch was sized for, and within [1, max_chunk].  The
// plan guarantees floor <= what the LDS holds for every team in the call; the
// clamps make the result safe even if a team's setting changed since then.
MRV_HD inline int query_chunk(int team_chunk, int lds_bytes, int lds_per_t, int chunk_floor, int max_chunk)
{
    int lds_fit = lds_per_t > 0 ? (lds_bytes - 64) / lds_per_t : max_chunk;
    int c = team_chunk < lds_fit ? team_chunk : lds_fit;
    if (c < chunk_floor) c = chunk_floor;
    if (c > max_chunk) c = max_chunk;
    return c < 1 ? 1 : c;
}

// Tiles of a query with horizon T (states) and tile length chunk.
MRV_HD inline long long tiles_of(long long T, int chunk) { return (T + chunk - 1) / chunk; }

// Bins of the tile-count histogram for a call: tile counts 0..tiles_of(max_T,
// chunk_floor), plus one spare for the descending scan.
inline long long tile_bins(long long max_T, int chunk_floor)
{
    return tiles_of(max_T, chunk_floor < 1 ? 1 : chunk_floor) + 2;
}

}  // namespace mrv
