// Host-side graph algorithms of the hierarchy set-up (see graph.cpp).
#pragma once
#include <cstdint>
#include <vector>

#include "common.h"

namespace slamg {

void strength_sets(const HCsr& N, double theta, int rule, int top_s, std::vector<int>& Sp, std::vector<int>& Si);
std::vector<char> rs_coarsen(const std::vector<int>& Sp, const std::vector<int>& Si, int n);
void interp_pattern(const std::vector<int>& Sp, const std::vector<int>& Si, const HCsr& N,
                    const std::vector<char>& is_c, int cap, std::vector<int>& ptr, std::vector<int>& fine_cols,
                    int& capped);
// values = false: the pattern only (T.v stays empty)
HCsr transpose(const HCsr& A, std::vector<int>* perm, bool values = true);
HCsr symbolic_product(const HCsr& L, const HCsr& R);
std::vector<int> greedy_row_colouring(const HCsr& A);
void colour_order(const std::vector<int>& colour, std::vector<int>& rows, std::vector<int>& cptr);
HCsr union_pattern(const HCsr& A, const HCsr& B);

}  // namespace slamg
