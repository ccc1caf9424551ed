// partition.hip -- the C-ABI entry point of the graph partitioner
// (partition.hpp): host code only, no device work.
#include <stdint.h>

#include <cmath>
#include <string>

#include "cggm.h"
#include "internal.hpp"
#include "partition.hpp"
#include "solver.hpp"

extern "C" int cggm_partition_graph(int64_t n, const int64_t *rowptr, const int32_t *col,
                                    int64_t nparts, double imbalance, int32_t *part,
                                    int64_t *cut) {
    return cggm::guarded([&] {
        using cggm::fail;
        if (n < 1 || n > INT32_MAX || nparts < 1 || nparts > n)
            fail(CGGM_EINVAL, "partition_graph: 1 <= nparts <= n < 2^31 is required");
        if (!(imbalance >= 0.0) || !std::isfinite(imbalance))
            fail(CGGM_EINVAL, "partition_graph: imbalance must be finite and >= 0");
        if (!rowptr || !part) fail(CGGM_EINVAL, "partition_graph: null pointer");
        if (rowptr[n] > 0 && !col) fail(CGGM_EINVAL, "partition_graph: null col");
        cggm::part::Graph g;
        if (!cggm::part::undirected(n, rowptr, col, g))
            fail(CGGM_EINVAL, "partition_graph: rowptr must start at 0 and not decrease, and "
                              "every column must lie in [0, n)");
        cggm::part::partition(g, nparts, imbalance, part);
        if (cut) *cut = cggm::part::edge_cut(g, part);
        return CGGM_OK;
    });
}
