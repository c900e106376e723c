// Internal interface of the Cartesian acquisition (cart.hip) for the plan code (nufft.hip).
#pragma once
#include "common.hpp"

namespace mrf {

struct CartOp {
  int N, L;
  const cf* tw;          // [N] exp(-2 pi i k / N)
  const uint8_t* mask;   // [L][N][N] 0/1
};

bool cart_supported(int N);
long cart_part_blocks(int N, int L);
mrf_status cart_fwd(const CartOp& op, const cf* img, cf* ksp, cf* T, const cf* smap, hipStream_t s);
mrf_status cart_resid(const CartOp& op, const cf* img, const cf* b, cf* r, cf* T, double* part, const cf* smap,
                      hipStream_t s);
mrf_status cart_adj(const CartOp& op, const cf* ksp, cf* img, cf* T, const cf* smap, int accumulate, hipStream_t s);

}  // namespace mrf
