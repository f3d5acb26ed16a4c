// CPU check of the tile order of the symmetric all-pairs launch (sym_tile_of,
// sym_tile_at, sym_index_of and sym_share_range in csrc/kernels.h, the
// functions the kernels call).  For every block count given on the command
// line it maps each workgroup of a whole-triangle launch to its tile and checks
// that the tiles are the upper triangle b1 <= b2 < nblk, each exactly once,
// that fewer than kSymXcds workgroups get no tile, and that sym_index_of
// inverts sym_tile_at; it checks that the shares of 1, 2, 3, 8 and 13 equal
// parts cover the triangle exactly once through launches of their own ranges;
// and it reports the most distinct blocks that the tiles of 96 consecutive
// workgroups of one XCD touch (the blocks its L2 holds at a time with 32 CUs
// of 3 workgroups).  Prints one line per block count and exits non-zero on the
// first violation.  The launches with the j chunks of each tile cut into 2 or 4 parts
// (sym_item_of) must run every (tile, part) exactly once.
#include "kernels.h"

#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

namespace {

// tiles of the launch over order range [t0, t0 + count), appended with their XCD
bool walk(int64_t nblk, int64_t t0, int64_t count, std::vector<char> &seen,
          std::vector<std::vector<int64_t>> *per_xcd, int64_t *idle)
{
    const int64_t grid = nbk::sym_grid(count);
    if (grid % nbk::kSymXcds != 0 || grid - count >= nbk::kSymXcds) {
        std::printf("nblk=%lld: grid %lld for %lld tiles\n", (long long)nblk, (long long)grid, (long long)count);
        return false;
    }
    for (int64_t wg = 0; wg < grid; ++wg) {
        int64_t b1 = -1, b2 = -1;
        if (!nbk::sym_tile_of(wg, nblk, t0, count, b1, b2)) {
            ++*idle;
            continue;
        }
        if (b1 < 0 || b2 < b1 || b2 >= nblk) {
            std::printf("nblk=%lld wg=%lld: tile (%lld, %lld) outside the triangle\n", (long long)nblk,
                        (long long)wg, (long long)b1, (long long)b2);
            return false;
        }
        const int64_t t = nbk::sym_index_of(b1, b2, nblk);
        if (t < t0 || t >= t0 + count) {
            std::printf("nblk=%lld: tile (%lld, %lld) has index %lld outside [%lld, %lld)\n", (long long)nblk,
                        (long long)b1, (long long)b2, (long long)t, (long long)t0, (long long)(t0 + count));
            return false;
        }
        char &s = seen[(size_t)(b1 * nblk + b2)];
        if (s) {
            std::printf("nblk=%lld: tile (%lld, %lld) twice\n", (long long)nblk, (long long)b1, (long long)b2);
            return false;
        }
        s = 1;
        if (per_xcd) (*per_xcd)[(size_t)(wg % nbk::kSymXcds)].push_back(b1 * nblk + b2);
    }
    return true;
}

}  // namespace

int main(int argc, char **argv)
{
    for (int a = 1; a < argc; ++a) {
        const int64_t nblk = std::atoll(argv[a]);
        const int64_t tiles = nbk::sym_tiles(nblk);
        // the order index and its inverse
        for (int64_t t = 0; t < tiles; ++t) {
            int64_t b1, b2;
            nbk::sym_tile_at(t, nblk, b1, b2);
            if (nbk::sym_index_of(b1, b2, nblk) != t) {
                std::printf("nblk=%lld: index %lld -> (%lld, %lld) -> %lld\n", (long long)nblk, (long long)t,
                            (long long)b1, (long long)b2, (long long)nbk::sym_index_of(b1, b2, nblk));
                return 1;
            }
        }
        // the whole triangle in one launch
        std::vector<char> seen((size_t)(nblk * nblk), 0);
        std::vector<std::vector<int64_t>> per_xcd(nbk::kSymXcds);
        int64_t idle = 0;
        if (!walk(nblk, 0, tiles, seen, &per_xcd, &idle)) return 1;
        int64_t count = 0;
        for (char s : seen) count += s;
        if (count != tiles) {
            std::printf("nblk=%lld: %lld of %lld tiles\n", (long long)nblk, (long long)count, (long long)tiles);
            return 1;
        }
        // j parts: every (tile, part) exactly once, the parts of a tile on one XCD next to
        // each other, fewer than kSymXcds idle workgroups
        for (int split : {2, 4}) {
            std::vector<char> seen_p((size_t)(nblk * nblk * split), 0);
            const int64_t grid = nbk::sym_grid(tiles * split);
            int64_t idle_p = 0;
            for (int64_t wg = 0; wg < grid; ++wg) {
                int64_t b1 = -1, b2 = -1;
                int h = -1;
                if (!nbk::sym_item_of(wg, nblk, 0, tiles, split, b1, b2, h)) {
                    ++idle_p;
                    continue;
                }
                char &c = seen_p[(size_t)((b1 * nblk + b2) * split + h)];
                if (b1 < 0 || b2 < b1 || b2 >= nblk || h < 0 || h >= split || c) {
                    std::printf("nblk=%lld split=%d: item (%lld, %lld, %d) invalid or twice\n", (long long)nblk,
                                split, (long long)b1, (long long)b2, h);
                    return 1;
                }
                c = 1;
                // the previous workgroup of this XCD ran the previous part of the same tile
                if (h > 0 && wg >= nbk::kSymXcds) {
                    int64_t p1, p2;
                    int ph;
                    if (!nbk::sym_item_of(wg - nbk::kSymXcds, nblk, 0, tiles, split, p1, p2, ph) || p1 != b1 ||
                        p2 != b2 || ph != h - 1) {
                        std::printf("nblk=%lld split=%d: parts of (%lld, %lld) not consecutive\n", (long long)nblk,
                                    split, (long long)b1, (long long)b2);
                        return 1;
                    }
                }
            }
            int64_t c = 0;
            for (char x : seen_p) c += x;
            if (c != tiles * split || idle_p >= nbk::kSymXcds) {
                std::printf("nblk=%lld split=%d: %lld of %lld items, %lld idle\n", (long long)nblk, split,
                            (long long)c, (long long)(tiles * split), (long long)idle_p);
                return 1;
            }
        }
        // shares, each in a launch of its own
        for (int64_t shares : {1, 2, 3, 8, 13}) {
            std::vector<char> seen_s((size_t)(nblk * nblk), 0);
            int64_t idle_s = 0, total = 0;
            for (int64_t sh = 0; sh < shares; ++sh) {
                int64_t t0, cnt;
                nbk::sym_share_range(nblk, sh, shares, t0, cnt);
                if (cnt < tiles / shares || cnt > tiles / shares + 1) {
                    std::printf("nblk=%lld: share %lld of %lld has %lld tiles\n", (long long)nblk, (long long)sh,
                                (long long)shares, (long long)cnt);
                    return 1;
                }
                total += cnt;
                if (!walk(nblk, t0, cnt, seen_s, nullptr, &idle_s)) return 1;
            }
            int64_t c = 0;
            for (char s : seen_s) c += s;
            if (c != tiles || total != tiles) {
                std::printf("nblk=%lld: %lld shares cover %lld of %lld tiles\n", (long long)nblk, (long long)shares,
                            (long long)c, (long long)tiles);
                return 1;
            }
        }
        int64_t worst = 0;
        for (const auto &v : per_xcd)
            for (size_t i = 0; i + 96 <= v.size() || (i == 0 && !v.empty()); i += 16) {
                std::set<int64_t> blocks;
                for (size_t k = i; k < v.size() && k < i + 96; ++k) {
                    blocks.insert(v[k] / nblk);
                    blocks.insert(v[k] % nblk);
                }
                worst = std::max<int64_t>(worst, (int64_t)blocks.size());
            }
        std::printf("nblk=%lld tiles=%lld grid=%lld idle=%lld window_blocks_max=%lld ok\n", (long long)nblk,
                    (long long)tiles, (long long)nbk::sym_grid(tiles), (long long)idle, (long long)worst);
    }
    return 0;
}
