// TIMEST reference oracle -- TEST INFRASTRUCTURE ONLY (see timest_oracle.h).
// Graph container shared by the oracle's own translation units.
#ifndef TIMEST_ORACLE_GRAPH_INTERNAL_H
#define TIMEST_ORACLE_GRAPH_INTERNAL_H

#include <cstdint>
#include <map>
#include <utility>
#include <vector>

struct OEdge {
    int32_t u, v;
    int64_t t;
};

// Sec. 4 keeps per-vertex in/out lists sorted by time; timestamps are shifted
// to start at 0.  Ties in time are broken by (u, v) so every edge has a
// canonical id (eid).  El_{u,v} is the multi-edge list (Def. "multi-edge list").
struct or_graph {
    int32_t n = 0;
    int64_t m = 0;
    int64_t shift = 0;
    int64_t T = 0;                                                   // largest shifted time
    std::vector<OEdge> e;                                            // indexed by eid
    std::vector<std::vector<int32_t>> out, in;                       // eids, increasing
    std::map<std::pair<int32_t, int32_t>, std::vector<int32_t>> el;  // El_{u,v}
};

#endif
