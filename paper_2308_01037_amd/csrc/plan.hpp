// Sizing of the diagonal gather's LDS table (host only, no HIP types, so it
// can be checked on its own).
#pragma once

#include <cstddef>
#include <cstdint>

namespace mcmf {

// A one-batch gather item keeps only its column entries in the table when
// its column chunks hold at most visits * kRestrictDen / kRestrictNum
// entries; it then claims at most that many keys (and at most n), which the
// plan's capacity covers whenever the whole row's walks fit one pass.
constexpr uint64_t kRestrictNum = 2, kRestrictDen = 1;

struct GatherPlan {
    int64_t cap;            // table slots (multiple of slots_per_bucket)
    int64_t walks_per_pass; // walks whose visits share one table fill
    int64_t distinct_max;   // most distinct states one pass can insert
    size_t lds_bytes;       // dynamic LDS: table + filter
    bool ok;                // cap > distinct_max and everything fits
};

// table_bytes: LDS available for the table (12 bytes per slot) plus the
// filter (filter_bytes).  Every state a pass visits must get its own slot
// and one slot must stay empty (the probe sequences end at an empty slot).
inline GatherPlan plan_gather(int64_t n, int64_t N, int K, size_t table_bytes, size_t filter_bytes,
                              int slots_per_bucket) {
    GatherPlan p = {};
    const int64_t sb = slots_per_bucket;
    if (K < 2 || N < 1 || n < 1 || table_bytes <= filter_bytes)
        return p;
    const int64_t cap_max = (static_cast<int64_t>((table_bytes - filter_bytes) / 12) / sb) * sb;
    const int64_t steps = K - 1;
    auto distinct_of = [&](int64_t walks) {
        const int64_t v = walks * steps;
        return v < n ? v : n;
    };
    int64_t wpp = N;
    // The worst case (every visit a new state) stays at or below 90% occupancy.
    if (distinct_of(N) * 10 > cap_max * 9) {
        wpp = (cap_max * 9 / 10) / steps;
        if (wpp < 1)
            wpp = 1;
    }
    const int64_t distinct = distinct_of(wpp);
    int64_t cap = distinct + distinct / 4 + 1; // 80% occupancy when it fits
    cap = ((cap + sb - 1) / sb) * sb;
    if (cap > cap_max)
        cap = cap_max;
    p.cap = cap;
    p.walks_per_pass = wpp;
    p.distinct_max = distinct;
    p.lds_bytes = 12 * static_cast<size_t>(cap) + filter_bytes;
    p.ok = cap >= sb && cap > distinct;
    return p;
}

} // namespace mcmf
