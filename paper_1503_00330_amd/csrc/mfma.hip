// FP32 matrix-core kernels for gfx950 (v_mfma_f32_16x16x4f32).
//
// The kernel distance of Eq. (1) is recast as a dense contraction: with
// Phi(z) = [z_a z_b (a <= b), z, 1] the activation of model j is
//   alpha * q_j = Phi(z) . w_j,   w_j = alpha [theta_j, -(D_j + D_j^T) c_j, c_j^T D_j c_j],
// alpha = -log2(e)/2, and the local prediction is y_j = [z, 1] . [b_j, beta0_j - b_j.c_j].
// A workgroup owns 16*MT samples (rows of the A operand, staged in LDS as
// lane-major fragments); its NW waves split the model tiles (16 models = the
// columns of one B operand, streamed from L2 as 1 KB coalesced loads).  Each
// lane folds its 4 rows x 1 column results into running softmax/Welford
// statistics (base-2 shift), which are merged across the 16 column lanes with
// cross-lane shuffles and across waves in LDS, in a fixed order.
// (PI^2-RH with LWPR dynamics, arXiv:1503.00330.)
#include "internal.hpp"

namespace pi2rh {

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int D>
struct Geo {
  static constexpr int NP = D * (D + 1) / 2;
  static constexpr int KQ = NP + D + 1;
  static constexpr int KQB = (KQ + 3) / 4;
  static constexpr int KY = D + 1;
  static constexpr int KYB = (KY + 3) / 4;
  static constexpr int KB = KQB + KYB;
  static constexpr int KB4 = (KB + 3) / 4;
};

// alpha = -log2(e) / 2
constexpr double kAlpha = -0.72134752044448170368;
constexpr float kPadAct = -1.0e30f;

// ----------------------------------------------------------------- fold
// One block per tile of 16 model slots.  Phase 1: one lane per model computes
// in double the derived vectors (h = -(D + D^T) c, kappa = c^T D c, the folded
// PLS map b and y0 = beta0 - b.c) into LDS; phase 2: every lane writes whole
// float4 fragments, coalesced.
constexpr int kFoldThreads = 256;

__global__ void __launch_bounds__(kFoldThreads) fold_mfma_kernel(ModelArgs m, MfmaLayout l,
                                                                 float *__restrict__ W,
                                                                 float *__restrict__ sig2) {
  __shared__ double hv[16][kMaxD], bv[16][kMaxD], kap[16], y0v[16];
  __shared__ int jcol[16];
  const int tile = blockIdx.x, d = m.d, R = m.R;
  const MfmaGeom g = MfmaGeom::make(d);
  int o = 0;
  while (o + 1 < m.n_out && tile >= l.tile_off[o + 1]) ++o;
  if (threadIdx.x < 16) {
    const int col = threadIdx.x;
    const int jloc = (tile - l.tile_off[o]) * 16 + col;
    const int j = jloc < m.L_off[o + 1] - m.L_off[o] ? m.L_off[o] + jloc : -1;
    jcol[col] = j;
    if (j >= 0) {
      const float *c = (const float *)m.centre + (size_t)j * d;
      const float *D = (const float *)m.metric + (size_t)j * d * d;
      const float *U = (const float *)m.proj_u + (size_t)j * R * d;
      const float *P = m.proj_p ? (const float *)m.proj_p + (size_t)j * R * d : U;
      const float *B = (const float *)m.beta + (size_t)j * (R + 1);
      double kappa = 0.0;
      for (int a = 0; a < d; ++a) {
        double h = 0.0;
        for (int b = 0; b < d; ++b) {
          h += ((double)D[a * d + b] + (double)D[b * d + a]) * (double)c[b];
          kappa += (double)c[a] * (double)D[a * d + b] * (double)c[b];
        }
        hv[col][a] = -h;
      }
      kap[col] = kappa;
      // y = beta0 + b.(z - c): b by reverse accumulation through the deflation chain
      double rb[kMaxD];
      for (int a = 0; a < d; ++a) rb[a] = 0.0;
      for (int r = R - 1; r >= 0; --r) {
        double pr = 0.0;
        for (int a = 0; a < d; ++a) pr += (double)P[r * d + a] * rb[a];
        const double sb = (double)B[r + 1] - pr;
        for (int a = 0; a < d; ++a) rb[a] += sb * (double)U[r * d + a];
      }
      double y0 = (double)B[0];
      for (int a = 0; a < d; ++a) {
        bv[col][a] = rb[a];
        y0 -= rb[a] * (double)c[a];
      }
      y0v[col] = y0;
      sig2[tile * 16 + col] = ((const float *)m.sigma2)[j];
    } else {
      sig2[tile * 16 + col] = 0.0f;
    }
  }
  __syncthreads();
  const int NE = g.KB4 * 64 * 4;
  float *dst = W + (size_t)tile * NE;
  for (int e = threadIdx.x; e < NE; e += blockDim.x) {
    const int comp = e & 3, lane = (e >> 2) & 63, kb4 = e >> 8;
    const int f = 4 * (4 * kb4 + comp) + lane / 16, col = lane & 15;
    const int j = jcol[col];
    float v = 0.0f;
    if (j < 0) {
      v = (f == g.NP + d) ? kPadAct : 0.0f;
    } else if (f < g.NP) {
      int a = 0, rem = f;
      while (rem >= d - a) {
        rem -= d - a;
        ++a;
      }
      const int b = a + rem;
      const float *D = (const float *)m.metric + (size_t)j * d * d;
      const double th = (a == b) ? (double)D[a * d + a] : (double)D[a * d + b] + (double)D[b * d + a];
      v = (float)(kAlpha * th);
    } else if (f < g.NP + d) {
      v = (float)(kAlpha * hv[col][f - g.NP]);
    } else if (f == g.NP + d) {
      v = (float)(kAlpha * kap[col]);
    } else if (f >= 4 * g.KQB && f < 4 * g.KQB + d) {
      v = (float)bv[col][f - 4 * g.KQB];
    } else if (f == 4 * g.KQB + d) {
      v = (float)y0v[col];
    }
    dst[e] = v;
  }
}

hipError_t launch_fold_mfma(int, const ModelArgs &m, const MfmaLayout &l, void *base, hipStream_t s) {
  float *W = (float *)base;
  float *sig = (float *)((char *)base + align_up(l.w_floats * 4, 256));
  hipLaunchKernelGGL(fold_mfma_kernel, dim3(l.n_tiles), dim3(kFoldThreads), 0, s, m, l, W, sig);
  return hipGetLastError();
}

static MfmaModel mfma_view(const MfmaLayout &l, const void *base) {
  MfmaModel md;
  md.W = (const float4 *)base;
  md.sig2 = (const float *)((const char *)base + align_up(l.w_floats * 4, 256));
  md.n_out = l.n_out;
  md.n_tiles = l.n_tiles;
  for (int o = 0; o <= kMaxOut; ++o) md.tile_off[o] = l.tile_off[o];
  return md;
}

// ------------------------------------------------------ shared mixture
template <int D, int MT, int NW>
struct MixSmem {
  static constexpr int ROWS = 16 * MT;
  float4 A[MT][Geo<D>::KB4][64];                 // A fragments, lane-major
  MixStat<float> part[NW][kMaxOut][ROWS];        // per-wave partial statistics
  float z[ROWS][D];
  float mean[ROWS][kMaxOut], var[ROWS][kMaxOut];
  unsigned char pa[Geo<D>::NP], pb[Geo<D>::NP];  // feature -> (a, b)
};

template <int D, int MT, int NW>
__device__ void mix_setup(MixSmem<D, MT, NW> &sm) {
  if (threadIdx.x == 0) {
    int f = 0;
    for (int a = 0; a < D; ++a)
      for (int b = a; b < D; ++b) {
        sm.pa[f] = (unsigned char)a;
        sm.pb[f] = (unsigned char)b;
        ++f;
      }
  }
}

// Stage 1 (all lanes): A fragments from sm.z; resets the partial statistics.
template <int D, int MT, int NW>
__device__ __forceinline__ void build_fragments(MixSmem<D, MT, NW> &sm) {
  using G = Geo<D>;
  constexpr int NE = MT * G::KB4 * 64 * 4;
  float *Af = (float *)&sm.A[0][0][0];
  for (int e = threadIdx.x; e < NE; e += NW * 64) {
    const int comp = e & 3, lane = (e >> 2) & 63, kb4 = (e >> 8) % G::KB4, mt = (e >> 8) / G::KB4;
    const int kb = 4 * kb4 + comp, f = 4 * kb + lane / 16, row = 16 * mt + (lane & 15);
    float v = 0.0f;
    if (f < G::NP) {
      v = sm.z[row][sm.pa[f]] * sm.z[row][sm.pb[f]];
    } else if (f < G::NP + D) {
      v = sm.z[row][f - G::NP];
    } else if (f == G::NP + D) {
      v = 1.0f;
    } else if (f >= 4 * G::KQB) {
      const int g = f - 4 * G::KQB;
      v = g < D ? sm.z[row][g] : (g == D ? 1.0f : 0.0f);
    }
    Af[e] = v;
  }
  MixStat<float> *pp = &sm.part[0][0][0];
  for (int i = threadIdx.x; i < NW * kMaxOut * MixSmem<D, MT, NW>::ROWS; i += NW * 64)
    pp[i] = mix_empty<float>();
}

__device__ __forceinline__ MixStat<float> shfl_xor_stat(const MixStat<float> &s, int mask) {
  MixStat<float> r;
  r.m = __shfl_xor(s.m, mask);
  r.Z = __shfl_xor(s.Z, mask);
  r.mu = __shfl_xor(s.mu, mask);
  r.M2 = __shfl_xor(s.M2, mask);
  r.S2 = __shfl_xor(s.S2, mask);
  return r;
}

// Stage 2 (each wave): its contiguous range of model tiles, one MFMA chain per
// tile; statistics flushed per output into sm.part[wave][o][row].
template <int D, int MT, int NW>
__device__ __forceinline__ void mixture_tiles(const MfmaModel &md, MixSmem<D, MT, NW> &sm) {
  using G = Geo<D>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  f32x4 A[MT][G::KB4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int q = 0; q < G::KB4; ++q) {
      const float4 v = sm.A[mt][q][lane];
      A[mt][q] = f32x4{v.x, v.y, v.z, v.w};
    }
  const int t0 = (int)((int64_t)wave * md.n_tiles / NW), t1 = (int)((int64_t)(wave + 1) * md.n_tiles / NW);
  if (t0 >= t1) return;
  int o = 0;
  while (o + 1 < md.n_out && t0 >= md.tile_off[o + 1]) ++o;
  MixStat<float> st[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) st[mt][r] = mix_empty<float>();

  auto flush = [&](int oo) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        MixStat<float> s = st[mt][r];
#pragma unroll
        for (int msk = 8; msk >= 1; msk >>= 1) s = mix_merge<true>(s, shfl_xor_stat(s, msk));
        if ((lane & 15) == 0) sm.part[wave][oo][16 * mt + 4 * (lane >> 4) + r] = s;
        st[mt][r] = mix_empty<float>();
      }
  };

  // Software pipeline over tiles with two B buffers: the loads of tile i+1
  // are issued before the MFMA chain of tile i, and scheduling barriers keep
  // the compiler from sinking them next to their use.
  // sigma^2 of the lane's model column travels with its tile (loads complete
  // in order, so a later load would make the wait drain the prefetch too).
  f32x4 B0[G::KB4], B1[G::KB4];
  float s2_0, s2_1;
  auto load_tile = [&](f32x4 (&Bd)[G::KB4], float &s2d, int tile) {
    const f32x4 *src = (const f32x4 *)md.W + (size_t)tile * G::KB4 * 64 + lane;
#pragma unroll
    for (int q = 0; q < G::KB4; ++q) Bd[q] = src[q * 64];
    s2d = md.sig2[tile * 16 + (lane & 15)];
  };
  auto compute_tile = [&](const f32x4 (&Bc)[G::KB4], float s2, int tile) {
    if (tile >= md.tile_off[o + 1]) {
      flush(o);
      while (tile >= md.tile_off[o + 1]) ++o;
    }
    f32x4 qa[MT], qb[MT], ya[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      qa[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
      qb[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
      ya[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    // two interleaved accumulators per row tile shorten the dependency chain
#pragma unroll
    for (int kb = 0; kb < G::KQB; ++kb)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        if (kb & 1)
          qb[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[mt][kb / 4][kb % 4], Bc[kb / 4][kb % 4],
                                                        qb[mt], 0, 0, 0);
        else
          qa[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[mt][kb / 4][kb % 4], Bc[kb / 4][kb % 4],
                                                        qa[mt], 0, 0, 0);
      }
#pragma unroll
    for (int kb = G::KQB; kb < G::KB; ++kb)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        ya[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[mt][kb / 4][kb % 4], Bc[kb / 4][kb % 4],
                                                      ya[mt], 0, 0, 0);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) mix_add<true>(st[mt][r], qa[mt][r] + qb[mt][r], ya[mt][r], s2);
  };

  load_tile(B0, s2_0, t0);
  for (int tile = t0; tile < t1; tile += 2) {
    if (tile + 1 < t1) load_tile(B1, s2_1, tile + 1);
    __builtin_amdgcn_sched_barrier(0);
    compute_tile(B0, s2_0, tile);
    __builtin_amdgcn_sched_barrier(0);
    if (tile + 1 >= t1) break;
    if (tile + 2 < t1) load_tile(B0, s2_0, tile + 2);
    __builtin_amdgcn_sched_barrier(0);
    compute_tile(B1, s2_1, tile + 1);
    __builtin_amdgcn_sched_barrier(0);
  }
  flush(o);
}

// Stage 3 (lanes < ROWS * n_out): fixed-order merge over waves.
template <int D, int MT, int NW>
__device__ __forceinline__ void merge_waves(MixSmem<D, MT, NW> &sm, int n_out) {
  constexpr int ROWS = MixSmem<D, MT, NW>::ROWS;
  for (int i = threadIdx.x; i < ROWS * n_out; i += NW * 64) {
    const int row = i % ROWS, o = i / ROWS;
    MixStat<float> s = sm.part[0][o][row];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = mix_merge<true>(s, sm.part[w][o][row]);
    mix_finish(s, &sm.mean[row][o], &sm.var[row][o]);
  }
}

// --------------------------------------------------------------- predict
template <int D, int MT, int NW>
__global__ void __launch_bounds__(NW * 64) predict_mfma_kernel(MfmaModel md, const float *__restrict__ Z,
                                                               int64_t N, float *__restrict__ mean,
                                                               float *__restrict__ var) {
  __shared__ MixSmem<D, MT, NW> sm;
  constexpr int ROWS = MixSmem<D, MT, NW>::ROWS;
  mix_setup(sm);
  const int64_t n0 = (int64_t)blockIdx.x * ROWS;
  for (int i = threadIdx.x; i < ROWS * D; i += NW * 64) {
    const int row = i / D, a = i % D;
    sm.z[row][a] = (n0 + row < N) ? Z[(n0 + row) * D + a] : 0.0f;
  }
  __syncthreads();
  build_fragments(sm);
  __syncthreads();
  mixture_tiles(md, sm);
  __syncthreads();
  merge_waves(sm, md.n_out);
  __syncthreads();
  for (int i = threadIdx.x; i < ROWS * md.n_out; i += NW * 64) {
    const int row = i / md.n_out, o = i % md.n_out;
    if (n0 + row < N) {
      mean[(n0 + row) * md.n_out + o] = sm.mean[row][o];
      var[(n0 + row) * md.n_out + o] = sm.var[row][o];
    }
  }
}

template <int D>
static hipError_t predict_mfma_d(const MfmaModel &md, const float *Z, int64_t N, float *mean,
                                 float *var, hipStream_t s) {
  constexpr int MT = 1, NW = 4;
  const int64_t nb = (N + 16 * MT - 1) / (16 * MT);
  hipLaunchKernelGGL((predict_mfma_kernel<D, MT, NW>), dim3((unsigned)nb), dim3(NW * 64), 0, s, md,
                     Z, N, mean, var);
  return hipGetLastError();
}

hipError_t launch_predict_mfma(const ModelArgs &m, const MfmaLayout &l, const void *base,
                               const void *Z, int64_t N, void *mean, void *var, hipStream_t s) {
  if (N == 0) return hipSuccess;
  const MfmaModel md = mfma_view(l, base);
  if (m.d == 16) return predict_mfma_d<16>(md, (const float *)Z, N, (float *)mean, (float *)var, s);
  if (m.d == 6) return predict_mfma_d<6>(md, (const float *)Z, N, (float *)mean, (float *)var, s);
  return hipErrorInvalidValue;
}

// --------------------------------------------------------------- rollout
template <int DYN>
struct Dims;
template <>
struct Dims<kDynPointMass2D> {
  static constexpr int NX = 4, NU = 2, NO = 2, D = 6;
};
template <>
struct Dims<kDynQuad12> {
  static constexpr int NX = 12, NU = 4, NO = 6, D = 16;
};

// One workgroup owns `spw` (<= 16*MT) sub-rollouts for the whole horizon.
// Per step: rows draw their noise and form z (A fragments), the waves run the
// model tiles, statistics are merged, and each row samples its accelerations,
// steps Euler and writes dt*q(x_{t+1}).
template <int DYN, int MT, int NW>
__global__ void __launch_bounds__(NW * 64) rollout_mfma_kernel(RolloutArgs<float> ra, MfmaModel md,
                                                               int spw) {
  using DD = Dims<DYN>;
  constexpr int D = DD::D, NX = DD::NX, NU = DD::NU, NO = DD::NO;
  constexpr int ROWS = 16 * MT;
  __shared__ MixSmem<D, MT, NW> sm;
  __shared__ float xs[ROWS][NX];
  __shared__ float xis[ROWS][8];
  __shared__ float obs[3 * kMaxObs];
  const ProbDev<float> &p = ra.p;
  mix_setup(sm);
  for (int i = threadIdx.x; i < 3 * p.n_obs; i += NW * 64) obs[i] = p.obs[i];
  const int row = threadIdx.x;
  const int64_t s = (int64_t)blockIdx.x * spw + row;
  const bool is_row = row < spw;
  const bool active = is_row && s < (int64_t)p.K * p.Ms;
  const uint32_t k = active ? (uint32_t)(s / p.Ms) : 0u, mm = active ? (uint32_t)(s % p.Ms) : 0u;
  const uint32_t it = *ra.iter;
  const uint32_t wc = stream_word(kTagCtrl, p.problem_id, it);
  const uint32_t wd = stream_word(kTagDyn, p.problem_id, it);
  if (row < ROWS)
    for (int a = 0; a < NX; ++a) xs[row][a] = ra.x0[a];
  for (int t = 0; t < p.T; ++t) {
    if (row < ROWS) {
      if (active) {
        float eps[4];
        normals<float, NU>(p.key0, p.key1, wc, k, 0u, (uint32_t)t, eps);
#pragma unroll
        for (int a = 0; a < NX; ++a) sm.z[row][a] = xs[row][a];
#pragma unroll
        for (int a = 0; a < NU; ++a) sm.z[row][NX + a] = ra.u_nom[t * NU + a] + p.noise_std[a] * eps[a];
        if (p.M > 0) normals<float, NO>(p.key0, p.key1, wd, k, mm, (uint32_t)t, xis[row]);
      } else {
#pragma unroll
        for (int a = 0; a < D; ++a) sm.z[row][a] = 0.0f;
      }
    }
    __syncthreads();
    build_fragments(sm);
    __syncthreads();
    mixture_tiles(md, sm);
    __syncthreads();
    merge_waves(sm, NO);
    __syncthreads();
    if (active) {
      float acc[NO], xn[NX], x[NX];
#pragma unroll
      for (int o = 0; o < NO; ++o)
        acc[o] = p.M > 0 ? sm.mean[row][o] + sqrtf(sm.var[row][o]) * xis[row][o] : sm.mean[row][o];
#pragma unroll
      for (int a = 0; a < NX; ++a) x[a] = xs[row][a];
      euler_step<float>(DYN, p.dt, x, acc, xn);
#pragma unroll
      for (int a = 0; a < NX; ++a) xs[row][a] = xn[a];
      ra.cost[s * p.T + t] = p.dt * state_cost<float>(p, obs, xn);
    }
  }
}

template <int DYN, int MT, int NW>
static hipError_t rollout_mfma_t(const RolloutArgs<float> &ra, const MfmaModel &md, int spw,
                                 hipStream_t s) {
  const int64_t n = (int64_t)ra.p.K * ra.p.Ms;
  const int64_t nb = (n + spw - 1) / spw;
  hipLaunchKernelGGL((rollout_mfma_kernel<DYN, MT, NW>), dim3((unsigned)nb), dim3(NW * 64), 0, s, ra,
                     md, spw);
  return hipGetLastError();
}

hipError_t launch_rollout_mfma(const RolloutArgs<float> &ra, const ModelArgs &m, const MfmaLayout &l,
                               const void *base, int tile_samples, int waves, hipStream_t s) {
  const MfmaModel md = mfma_view(l, base);
  const int spw = tile_samples;
  if (ra.p.dyn == kDynQuad12) {
    if (waves == 8) {
      if (spw <= 16) return rollout_mfma_t<kDynQuad12, 1, 8>(ra, md, spw, s);
      return rollout_mfma_t<kDynQuad12, 2, 8>(ra, md, spw, s);
    }
    if (spw <= 16) return rollout_mfma_t<kDynQuad12, 1, 4>(ra, md, spw, s);
    return rollout_mfma_t<kDynQuad12, 2, 4>(ra, md, spw, s);
  }
  if (spw <= 16) return rollout_mfma_t<kDynPointMass2D, 1, 4>(ra, md, spw, s);
  return rollout_mfma_t<kDynPointMass2D, 2, 4>(ra, md, spw, s);
}

}  // namespace pi2rh
