// CPU check of the tile order of the symmetric all-pairs launch (sym_tile_of in
// csrc/kernels.h, the function the kernel calls).  For every block count given
// on the command line it maps each workgroup of sym_grid(nblk) to its tile and
// checks that the tiles are the upper triangle b1 <= b2 < nblk, each exactly
// once, that fewer than kSymXcds workgroups get no tile, and it reports the most
// distinct blocks that the tiles of 96 consecutive workgroups of one XCD touch
// (the blocks its L2 holds at a time with 32 CUs of 3 workgroups).  Prints one
// line per block count and exits non-zero on the first violation.
#include "kernels.h"

#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

int main(int argc, char **argv)
{
    for (int a = 1; a < argc; ++a) {
        const int64_t nblk = std::atoll(argv[a]);
        const int64_t grid = nbk::sym_grid(nblk), tiles = nbk::sym_tiles(nblk);
        std::vector<char> seen((size_t)(nblk * nblk), 0);
        int64_t idle = 0, worst = 0;
        std::vector<std::vector<int64_t>> per_xcd(nbk::kSymXcds);
        for (int64_t wg = 0; wg < grid; ++wg) {
            int64_t b1 = -1, b2 = -1;
            if (!nbk::sym_tile_of(wg, nblk, b1, b2)) {
                ++idle;
                continue;
            }
            if (b1 < 0 || b2 < b1 || b2 >= nblk) {
                std::printf("nblk=%lld wg=%lld: tile (%lld, %lld) outside the triangle\n", (long long)nblk,
                            (long long)wg, (long long)b1, (long long)b2);
                return 1;
            }
            char &s = seen[(size_t)(b1 * nblk + b2)];
            if (s) {
                std::printf("nblk=%lld: tile (%lld, %lld) twice\n", (long long)nblk, (long long)b1, (long long)b2);
                return 1;
            }
            s = 1;
            per_xcd[(size_t)(wg % nbk::kSymXcds)].push_back(b1 * nblk + b2);
        }
        int64_t count = 0;
        for (char s : seen) count += s;
        if (count != tiles || idle >= nbk::kSymXcds || grid % nbk::kSymXcds != 0) {
            std::printf("nblk=%lld: %lld of %lld tiles, %lld idle workgroups\n", (long long)nblk, (long long)count,
                        (long long)tiles, (long long)idle);
            return 1;
        }
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
                    (long long)tiles, (long long)grid, (long long)idle, (long long)worst);
    }
    return 0;
}
