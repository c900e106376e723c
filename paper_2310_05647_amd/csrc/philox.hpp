// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC'11), written from its published definition: ten rounds of two 32x32 ->
// 64-bit multiplies with the Weyl key schedule. Shared by the kernels that draw random numbers.
#pragma once

namespace mrf {

struct u4 {
  unsigned x, y, z, w;
};

__device__ inline u4 philox(u4 c, unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
    const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
    const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
    c = u4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// uint32 -> (0, 1): (u + 1/2) 2^-32
__device__ inline float u01(unsigned u) { return ((float)u + 0.5f) * 2.3283064365386963e-10f; }

}  // namespace mrf
