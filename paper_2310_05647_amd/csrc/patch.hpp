// Patch lattice shared by the Laplacian, graph and LLR kernels (Sec. III-A, III-B).
//
// Patches are p x p with stride s, origins (a s, b s) for a, b in [0, n1), n1 = (N - p)/s + 1,
// numbered i = a n1 + b (raster order). The kernels require p % s == 0 and (N - p) % s == 0,
// so the image splits into (N/s)^2 "cells" of s x s pixels, and every pixel of a cell lies in
// the same patches: cell (cy, cx) is covered by the patches a in [cy - p/s + 1, cy] and
// b in [cx - p/s + 1, cx] (clipped to the lattice).
#pragma once
#include "common.hpp"

namespace mrf {

struct PatchGeom {
  int N, p, s, n1, Np, nc, ppc;  // ppc = p / s, nc = N / s cells per side
};

inline bool make_geom(int N, int p, int s, PatchGeom* g) {
  if (N <= 0 || p <= 0 || s <= 0 || p > N || p % s != 0 || (N - p) % s != 0) return false;
  g->N = N; g->p = p; g->s = s;
  g->n1 = (N - p) / s + 1;
  g->Np = g->n1 * g->n1;
  g->nc = N / s;
  g->ppc = p / s;
  return true;
}

// Covering patch range of cell coordinate c along one axis.
__host__ __device__ inline void cover_range(const PatchGeom& g, int c, int& lo, int& hi) {
  lo = c - g.ppc + 1;
  if (lo < 0) lo = 0;
  hi = c < g.n1 - 1 ? c : g.n1 - 1;
}

__host__ __device__ inline int coverage_1d(const PatchGeom& g, int c) {
  int lo, hi;
  cover_range(g, c, lo, hi);
  return hi - lo + 1;
}

}  // namespace mrf
