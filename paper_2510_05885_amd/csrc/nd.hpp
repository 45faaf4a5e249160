// nd.hpp — nested-dissection ordering used by the symbolic analysis.
#pragma once
#include <cstdint>
#include <vector>

namespace ncl {

// Fill-reducing elimination order of a symmetric graph (CSR adjacency without
// self loops): indistinguishable vertices are merged, the merged graph is
// dissected recursively (separators last) down to `leaf` vertices, leaves are
// ordered by minimum degree.  Returns perm[k] = vertex eliminated k-th.
std::vector<int> nd_order(int N, const std::vector<int64_t>& xadj, const std::vector<int>& adj,
                          int leaf, uint64_t seed);

}  // namespace ncl
