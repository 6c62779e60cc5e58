// Work table of the inter-body sum (host C++ only, no HIP: also compiled by the
// CPU tests).  The sum over sources on other bodies (Sec. 3.3, the blocks
// A_pq with p != q) is cut into work items: every body-aligned tile of at most
// `tile` consecutive target nodes, against `splits` chunks of the source units
// (nodes, azimuthal rings or 32-node blocks) that belong to other bodies.  The
// units of all bodies are numbered consecutively, body by body; an item's
// sources are the two unit ranges [s0, s1) (before the target's body) and
// [s2, s3) (after it), so no pair needs a mask.  Item `slot` s of a tile
// writes partial sum s; the splits of one tile cover every other body's unit
// exactly once.
#pragma once

#include <algorithm>
#include <cstdint>
#include <limits>
#include <stdexcept>
#include <vector>

namespace axs {

struct IBWork {
    int32_t t0, tn;           // first target node, number of targets
    int32_t s0, s1, s2, s3;   // source unit ranges [s0, s1) and [s2, s3)
    int32_t slot, pad;        // partial-sum slot (the split index)
};

struct WorkBody {
    int64_t node_off, nodes;   // the body's target nodes [node_off, node_off + nodes)
    int64_t unit_off, units;   // its source units [unit_off, unit_off + units)
};

// total_units: units of all bodies; tile >= 1; splits >= 1.  Throws
// std::invalid_argument for bad sizes and std::length_error where node or
// unit indices would not fit the items' 32-bit fields.
inline std::vector<IBWork> build_work_table(const std::vector<WorkBody> &bodies, int64_t total_units, int tile,
                                            int splits) {
    if (tile < 1 || splits < 1 || total_units < 0) throw std::invalid_argument("work table: bad tile or splits");
    constexpr int64_t lim = std::numeric_limits<int32_t>::max();
    if (total_units > lim) throw std::length_error("work table: more than 2^31 - 1 source units");
    std::vector<IBWork> out;
    for (const WorkBody &b : bodies) {
        if (b.nodes < 0 || b.units < 0 || b.unit_off < 0 || b.unit_off + b.units > total_units)
            throw std::invalid_argument("work table: body units out of range");
        if (b.node_off < 0 || b.node_off + b.nodes > lim)
            throw std::length_error("work table: more than 2^31 - 1 target nodes");
        const int64_t others = total_units - b.units;
        const int64_t chunk = (std::max<int64_t>(others, 1) + splits - 1) / splits;
        for (int64_t t0 = 0; t0 < b.nodes; t0 += tile) {
            for (int s = 0; s < splits; ++s) {
                IBWork w{};
                w.t0 = (int32_t)(b.node_off + t0);
                w.tn = (int32_t)std::min<int64_t>(tile, b.nodes - t0);
                // chunk s of the other bodies' units in a numbering that skips
                // the target's body: virtual v < unit_off is unit v, v >=
                // unit_off is unit v + units
                const int64_t v0 = std::min<int64_t>(others, (int64_t)s * chunk);
                const int64_t v1 = std::min<int64_t>(others, v0 + chunk);
                const int64_t a0 = v0, a1 = std::max(a0, std::min<int64_t>(v1, b.unit_off));
                const int64_t c0 = std::max<int64_t>(v0, b.unit_off), c1 = std::max(c0, v1);
                w.s0 = (int32_t)a0;
                w.s1 = (int32_t)a1;
                w.s2 = (int32_t)(c0 + b.units);
                w.s3 = (int32_t)(c1 + b.units);
                w.slot = s;
                out.push_back(w);
            }
        }
    }
    return out;
}

}  // namespace axs
