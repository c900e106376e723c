// Device-resident dictionary shared by the subspace match, the full-length match and the
// reconstruction driver (Sec. II-B, eqs. (3)-(5)).
#pragma once
#include "common.hpp"

struct mrf_dict_s {
  int M, L, r, nparam, ntile;
  float* lut;        // [M][nparam]
  float* norms;      // [M] ||d_m|| (computed in double)
  mrf::cf* dhr;      // [M][r] (d_m V) / ||d_m||
  float* bpk;        // [ntile][10][64] MFMA B operands of the subspace match (r <= 10)
  mrf::cf* V;        // [L][r]
  mrf::cf* dn;       // [M][L] unit-norm atoms (full-length matching and the FP32 re-rank)
  int Lp;            // L rounded up to a multiple of 128: length of each part of the rows below
  uint16_t* d16;     // [M][2 Lp] unit-norm atoms in BF16, real parts then imaginary parts
  uint16_t* d16lo;   // [M][2 Lp] the BF16 remainders (atom - BF16 atom, rounded to BF16)
  uint8_t* d8;       // [M][2 Lp] the same in FP8 (OCP E4M3), scaled per row
  float* s8;         // [M] the FP8 row scales (value = code * s8[m])
};

namespace mrf {
// BF16 (with remainders) and FP8 row copies of `rows` complex rows of length L into [rows][2 Lp] split layout.
mrf_status quantise_rows(const cf* src, int rows, int L, int Lp, uint16_t* d16, uint16_t* d16lo, uint8_t* d8,
                         float* s8, hipStream_t s);
}  // namespace mrf
