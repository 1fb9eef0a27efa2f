// Host symbolic analysis of a symmetric pattern for supernodal Cholesky.
#pragma once

#include <cstdint>
#include <vector>

#include "opf.h"

namespace opf {

struct Symbolic {
    int n = 0;
    int nsuper = 0;
    std::vector<int32_t> perm, iperm;   // perm[k] = original index of pivot k
    std::vector<int32_t> parent;        // elimination tree in pivot order
    std::vector<int32_t> colcount;      // nonzeros per column of L (incl. diagonal)
    std::vector<int32_t> snode_ptr;     // first pivot of each supernode [nsuper+1]
    std::vector<int32_t> col2sn;        // pivot -> supernode
    std::vector<int32_t> sparent;       // supernodal tree
    std::vector<int64_t> rows_ptr;      // [nsuper+1]
    std::vector<int32_t> rows_flat;     // row indices of each supernode (own columns first, then ascending)
};

std::vector<int32_t> min_degree_order(int n, const std::vector<int32_t>& colptr, const std::vector<int32_t>& rowind,
                                      double dense_frac, int32_t dense_abs);
Symbolic analyze_pattern(int n, const std::vector<int32_t>& colptr, const std::vector<int32_t>& rowind,
                         const chol_options& o);

}  // namespace opf
