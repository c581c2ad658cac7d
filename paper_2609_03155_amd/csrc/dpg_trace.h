// Host numbering of the global trace unknowns and CSR structure of the
// condensed system (internal to the library; the C ABI is include/dpg.h).
#pragma once

#include <cstdint>
#include <vector>

namespace dpg {

// glob[toff[c] + q]: global id of local trace function q of cell c (Ehat then
// Hhat, 24 r_c^2 in all), -1 where removed or constrained.  Throws
// std::invalid_argument when cells disagree on edge directions or face axes.
void trace_numbering(const int64_t* cells, const int8_t* face_kind, const int8_t* degree, int64_t n,
                     std::vector<int64_t>& toff, std::vector<int64_t>& glob, int64_t& n_dofs);

// CSR structure of A = sum_K P_K^T A_K P_K (columns ascending) and, per
// nonzero, the positions of its contributions in the concatenated cell
// matrices (A_off[c] + b n_t + a for A_K(a, b), column-major); per unknown,
// the positions of its right-hand-side contributions (b_off[c] + a).
void trace_csr(const std::vector<int64_t>& toff, const std::vector<int64_t>& glob, const std::vector<int64_t>& A_off,
               const std::vector<int64_t>& b_off, int64_t n_dofs, std::vector<int64_t>& row_ptr,
               std::vector<int32_t>& col, std::vector<int64_t>& contrib_ptr, std::vector<int64_t>& contrib,
               std::vector<int64_t>& rhs_ptr, std::vector<int64_t>& rhs_contrib);

}  // namespace dpg
