// Direct-form (VALU) building blocks shared by the direct kernels and the
// adjoint: the folded per-model record, its evaluation at an input, and the
// per-dynamics dimensions.  (PI^2-RH with LWPR dynamics, arXiv:1503.00330.)
#pragma once

#include "internal.hpp"

namespace pi2rh {

// ------------------------------------------------------- direct mixture
// Kernel distance and local prediction of one folded record at input z.
template <typename Real, int D>
__device__ __forceinline__ void eval_record(const Real *__restrict__ r, const Real (&z)[D], Real &q,
                                            Real &y) {
  Real dl[D];
#pragma unroll
  for (int a = 0; a < D; ++a) dl[a] = z[a] - r[a];
  const Real *th = r + D;
  q = 0;
  int idx = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    Real row = 0;
#pragma unroll
    for (int b = a; b < D; ++b) row += th[idx++] * dl[b];
    q += dl[a] * row;
  }
  const Real *bb = th + D * (D + 1) / 2;
  y = bb[D];
#pragma unroll
  for (int a = 0; a < D; ++a) y += bb[a] * dl[a];
}

template <typename Real, int D>
constexpr int rec_stride() {
  return D + D * (D + 1) / 2 + D + 2;
}

// Models staged per LDS tile (about 32 KB of records).
template <typename Real, int D>
constexpr int tile_models() {
  return (32768 / (int)(rec_stride<Real, D>() * sizeof(Real))) > 0
             ? (32768 / (int)(rec_stride<Real, D>() * sizeof(Real)))
             : 1;
}

// Every lane of the block evaluates Eq. (1) for its own input z against all
// models of all outputs; mean/var of output o land in out[o], out[kMaxOut+o]
// (per-lane LDS row).  Block-synchronous: every lane of the block must call.
template <typename Real, int D>
__device__ void direct_mixture(const ModelArgs &m, const Real *__restrict__ rec, const Real (&z)[D],
                               Real *tile, Real *out) {
  constexpr int RS = rec_stride<Real, D>();
  constexpr int TM = tile_models<Real, D>();
  for (int o = 0; o < m.n_out; ++o) {
    MixStat<Real> st = mix_empty<Real>();
    for (int j0 = m.L_off[o]; j0 < m.L_off[o + 1]; j0 += TM) {
      const int nj = min(TM, m.L_off[o + 1] - j0);
      __syncthreads();
      for (int i = threadIdx.x; i < nj * RS; i += blockDim.x) tile[i] = rec[(size_t)j0 * RS + i];
      __syncthreads();
      for (int jj = 0; jj < nj; ++jj) {
        Real q, y;
        eval_record<Real, D>(tile + jj * RS, z, q, y);
        mix_add<false>(st, (Real)-0.5 * q, y, tile[jj * RS + RS - 1]);
      }
    }
    mix_finish(st, &out[o], &out[kMaxOut + o]);
  }
}

// Mixture statistics of the lane `mask` away (xor) in the wave.
template <typename Real>
__device__ __forceinline__ MixStat<Real> shfl_stat(const MixStat<Real> &s, int mask) {
  MixStat<Real> r;
  r.m = __shfl_xor(s.m, mask);
  r.Z = __shfl_xor(s.Z, mask);
  r.mu = __shfl_xor(s.mu, mask);
  r.M2 = __shfl_xor(s.M2, mask);
  r.S2 = __shfl_xor(s.S2, mask);
  return r;
}

template <int DYN>
struct DynDims;
template <>
struct DynDims<kDynPointMass2D> {
  static constexpr int NX = 4, NU = 2, NO = 2, D = 6;
};
template <>
struct DynDims<kDynQuad12> {
  static constexpr int NX = 12, NU = 4, NO = 6, D = 16;
};
template <>
struct DynDims<kDynQuadHybrid> {
  static constexpr int NX = 9, NU = 4, NO = 3, D = 4;
};


}  // namespace pi2rh
