// CPU check of the inter-body work table (paper_1406_0236_amd/csrc/worktable.h):
// for seeded random bodies, tile sizes and split counts, the tiles of every
// body partition its target nodes, every tile has one item per split slot,
// and the splits of a tile cover each unit of the other bodies exactly once
// and no unit of its own body.  Bad sizes raise.  Prints "ok <cases>".
#include <cstdio>
#include <map>
#include <random>
#include <stdexcept>
#include <utility>
#include <vector>

#include "../../paper_1406_0236_amd/csrc/worktable.h"

using axs::IBWork;
using axs::WorkBody;

static int fail(const char *what, int cse) {
    std::printf("FAIL case %d: %s\n", cse, what);
    return 1;
}

int main() {
    std::mt19937_64 rng(20140601);
    const int tiles[] = {1, 7, 64, 128, 256, 512};
    const int splits_[] = {1, 2, 3, 16, 64};
    int cases = 0;
    for (int it = 0; it < 400; ++it) {
        const int nb = 1 + (int)(rng() % 12);
        const int kind = (int)(rng() % 3);   // units: nodes, rings (NF nodes each), 32-node blocks
        std::vector<WorkBody> bodies;
        int64_t noff = 0, uoff = 0;
        for (int b = 0; b < nb; ++b) {
            const int64_t nf = 1 + 2 * (int64_t)(rng() % 8);
            const int64_t ng = (rng() % 5 == 0) ? 0 : 1 + (int64_t)(rng() % 60);
            const int64_t n = ng * nf;
            const int64_t u = kind == 0 ? n : kind == 1 ? ng : (n + 31) / 32;
            bodies.push_back(WorkBody{noff, n, uoff, u});
            noff += n;
            uoff += u;
        }
        const int64_t U = uoff;
        const int tile = tiles[rng() % 6], splits = splits_[rng() % 5];
        const std::vector<IBWork> w = axs::build_work_table(bodies, U, tile, splits);
        ++cases;
        // group by tile
        std::map<std::pair<int, int>, std::vector<IBWork>> by_tile;
        for (const IBWork &x : w) by_tile[{x.t0, x.tn}].push_back(x);
        size_t expect_items = 0;
        for (const WorkBody &b : bodies) expect_items += (size_t)((b.nodes + tile - 1) / tile) * splits;
        if (w.size() != expect_items) return fail("item count", cases);
        for (const WorkBody &b : bodies) {
            // tiles partition [node_off, node_off + nodes)
            int64_t next = b.node_off;
            for (const auto &kv : by_tile) {
                const int t0 = kv.first.first, tn = kv.first.second;
                if (t0 < b.node_off || t0 >= b.node_off + b.nodes) continue;
                if (t0 != next) return fail("tiles not contiguous", cases);
                if (tn < 1 || tn > tile || t0 + tn > b.node_off + b.nodes) return fail("tile size", cases);
                next = t0 + tn;
                const std::vector<IBWork> &items = kv.second;
                if ((int)items.size() != splits) return fail("items per tile", cases);
                std::vector<int> slot_seen(splits, 0), cover(U, 0);
                for (const IBWork &x : items) {
                    if (x.slot < 0 || x.slot >= splits || slot_seen[x.slot]++) return fail("slots", cases);
                    // a non-empty range lies on its side of the target's body
                    if (x.s0 < 0 || x.s1 < x.s0 || (x.s1 > x.s0 && x.s1 > b.unit_off))
                        return fail("range before body", cases);
                    if (x.s3 < x.s2 || x.s3 > U || (x.s3 > x.s2 && x.s2 < b.unit_off + b.units))
                        return fail("range after body", cases);
                    for (int u = x.s0; u < x.s1; ++u) ++cover[u];
                    for (int u = x.s2; u < x.s3; ++u) ++cover[u];
                }
                for (int64_t u = 0; u < U; ++u) {
                    const bool own = u >= b.unit_off && u < b.unit_off + b.units;
                    if (cover[u] != (own ? 0 : 1)) return fail("source coverage", cases);
                }
            }
            if (next != b.node_off + b.nodes) return fail("tiles do not reach the body's end", cases);
        }
    }
    // bad arguments
    int raised = 0;
    try {
        axs::build_work_table({WorkBody{0, 10, 0, 10}}, 10, 0, 1);
    } catch (const std::invalid_argument &) {
        ++raised;
    }
    try {
        axs::build_work_table({WorkBody{0, 10, 0, 10}}, 10, 64, 0);
    } catch (const std::invalid_argument &) {
        ++raised;
    }
    try {
        axs::build_work_table({WorkBody{0, 10, 5, 10}}, 10, 64, 1);
    } catch (const std::invalid_argument &) {
        ++raised;
    }
    try {
        axs::build_work_table({WorkBody{0, 10, 0, 10}}, (int64_t)1 << 32, 64, 1);
    } catch (const std::length_error &) {
        ++raised;
    }
    try {
        axs::build_work_table({WorkBody{((int64_t)1 << 31) - 5, 10, 0, 10}}, 10, 64, 1);
    } catch (const std::length_error &) {
        ++raised;
    }
    if (raised != 5) return fail("bad arguments must raise", cases);
    std::printf("ok %d\n", cases);
    return 0;
}
