// Direct-form (VALU) kernels for float and double: model fold, LWPR
// prediction, sampled rollouts, sub-rollout averaging, the path-integral
// update and the receding-horizon shift.  One lane evaluates one input
// against every local model; model records are staged through LDS tiles and
// read as broadcasts.  (PI^2-RH with LWPR dynamics, arXiv:1503.00330.)
#include <algorithm>

#include "direct.hpp"

namespace pi2rh {

// ----------------------------------------------------------------- fold
// One block per 16 local models.  One lane per model folds the PLS chain
// (Sec. 2) into y = beta_0 + b . (z - c) -- b is the derivative of y w.r.t.
// the centred input, accumulated backwards through the deflation steps in
// double -- then all lanes write the 16 contiguous records, coalesced:
// [c | theta (upper triangle of D + D^T, diagonal D_aa) | b | beta_0 | sigma^2].
template <typename Real>
__global__ void __launch_bounds__(256) fold_direct_kernel(ModelArgs m, Real *__restrict__ rec) {
  __shared__ double bv[16][kMaxD];
  const int j0 = blockIdx.x * 16, d = m.d, R = m.R, RS = d + d * (d + 1) / 2 + d + 2;
  const int nj = min(16, m.Ltot - j0);
  if ((int)threadIdx.x < nj) {
    const int j = j0 + threadIdx.x;
    const Real *U = (const Real *)m.proj_u + (size_t)j * R * d;
    const Real *P = m.proj_p ? (const Real *)m.proj_p + (size_t)j * R * d : U;
    const Real *B = (const Real *)m.beta + (size_t)j * (R + 1);
    double rb[kMaxD];
    for (int a = 0; a < d; ++a) rb[a] = 0.0;
    for (int r = R - 1; r >= 0; --r) {
      double pr = 0.0;
      for (int a = 0; a < d; ++a) pr += (double)P[r * d + a] * rb[a];
      const double sb = (double)B[r + 1] - pr;
      for (int a = 0; a < d; ++a) rb[a] += sb * (double)U[r * d + a];
    }
    for (int a = 0; a < d; ++a) bv[threadIdx.x][a] = rb[a];
  }
  __syncthreads();
  const int np = d * (d + 1) / 2;
  for (int e = threadIdx.x; e < nj * RS; e += blockDim.x) {
    const int jj = e / RS, f = e % RS, j = j0 + jj;
    Real v;
    if (f < d) {
      v = ((const Real *)m.centre)[(size_t)j * d + f];
    } else if (f < d + np) {
      int a = 0, rem = f - d;
      while (rem >= d - a) {
        rem -= d - a;
        ++a;
      }
      const int b = a + rem;
      const Real *D = (const Real *)m.metric + (size_t)j * d * d;
      v = (a == b) ? D[a * d + a] : D[a * d + b] + D[b * d + a];
    } else if (f < d + np + d) {
      v = (Real)bv[jj][f - d - np];
    } else if (f == d + np + d) {
      v = ((const Real *)m.beta)[(size_t)j * (R + 1)];
    } else {
      v = ((const Real *)m.sigma2)[j];
    }
    rec[(size_t)j0 * RS + e] = v;
  }
}

hipError_t launch_fold_direct(int dtype, const ModelArgs &m, void *rec, hipStream_t s) {
  const int nb = (m.Ltot + 15) / 16;
  if (dtype == PI_F64)
    hipLaunchKernelGGL(fold_direct_kernel<double>, dim3(nb), dim3(256), 0, s, m, (double *)rec);
  else
    hipLaunchKernelGGL(fold_direct_kernel<float>, dim3(nb), dim3(256), 0, s, m, (float *)rec);
  return hipGetLastError();
}

template <typename Real, int D>
__global__ void __launch_bounds__(128) predict_direct_kernel(ModelArgs m, const Real *__restrict__ rec,
                                                             const Real *__restrict__ Z, int64_t N,
                                                             Real *__restrict__ mean,
                                                             Real *__restrict__ var) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Real *tile = (Real *)smem_raw;
  Real *out = tile + tile_models<Real, D>() * rec_stride<Real, D>() + threadIdx.x * 2 * kMaxOut;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Real z[D];
#pragma unroll
  for (int a = 0; a < D; ++a) z[a] = n < N ? Z[n * D + a] : (Real)0;
  direct_mixture<Real, D>(m, rec, z, tile, out);
  if (n < N)
    for (int o = 0; o < m.n_out; ++o) {
      mean[n * m.n_out + o] = out[o];
      var[n * m.n_out + o] = out[kMaxOut + o];
    }
}

template <typename Real, int D>
static hipError_t predict_direct_d(const ModelArgs &m, const void *rec, const void *Z, int64_t N,
                                   void *mean, void *var, hipStream_t s) {
  const size_t sh = (size_t)(tile_models<Real, D>() * rec_stride<Real, D>() + 128 * 2 * kMaxOut) *
                    sizeof(Real);
  const int64_t nb = (N + 127) / 128;
  hipLaunchKernelGGL((predict_direct_kernel<Real, D>), dim3((unsigned)nb), dim3(128), sh, s, m,
                     (const Real *)rec, (const Real *)Z, N, (Real *)mean, (Real *)var);
  return hipGetLastError();
}

template <typename Real>
static hipError_t predict_direct_t(const ModelArgs &m, const void *rec, const void *Z, int64_t N,
                                   void *mean, void *var, hipStream_t s) {
  switch (m.d) {
#define PI_CASE(DD) \
  case DD:          \
    return predict_direct_d<Real, DD>(m, rec, Z, N, mean, var, s);
    PI_CASE(1) PI_CASE(2) PI_CASE(3) PI_CASE(4) PI_CASE(5) PI_CASE(6) PI_CASE(7) PI_CASE(8)
    PI_CASE(9) PI_CASE(10) PI_CASE(11) PI_CASE(12) PI_CASE(13) PI_CASE(14) PI_CASE(15) PI_CASE(16)
#undef PI_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_predict_direct(int dtype, const ModelArgs &m, const void *rec, const void *Z,
                                 int64_t N, void *mean, void *var, hipStream_t s) {
  if (N == 0) return hipSuccess;
  return dtype == PI_F64 ? predict_direct_t<double>(m, rec, Z, N, mean, var, s)
                         : predict_direct_t<float>(m, rec, Z, N, mean, var, s);
}

// One lane per sub-rollout (k, m): every step draws eps_{k,t} (shared by the
// sub-rollouts of k) and xi_{k,m,t}, evaluates Eq. (1) at z = [x ; u_nom + eps],
// samples the accelerations, steps Euler and writes dt * q(x_{t+1}).
template <typename Real, int DYN>
__global__ void __launch_bounds__(128) rollout_direct_kernel(RolloutArgs<Real> ra, ModelArgs m,
                                                             const Real *__restrict__ rec) {
  using DD = DynDims<DYN>;
  constexpr int D = DD::D, NX = DD::NX, NU = DD::NU, NO = DD::NO;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Real *tile = (Real *)smem_raw;
  Real *outb = tile + tile_models<Real, D>() * rec_stride<Real, D>();
  Real *out = outb + threadIdx.x * 2 * kMaxOut;
  Real *obs = outb + blockDim.x * 2 * kMaxOut;
  const ProbDev<Real> &p = ra.p;
  for (int i = threadIdx.x; i < 3 * p.n_obs; i += blockDim.x) obs[i] = p.obs[i];
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = s < (int64_t)p.K * p.Ms;
  const uint32_t k = (uint32_t)(s / p.Ms), mm = (uint32_t)(s % p.Ms);
  const uint32_t it = *ra.iter;
  const uint32_t wc = stream_word(kTagCtrl, p.problem_id, it);
  const uint32_t wd = stream_word(kTagDyn, p.problem_id, it);
  Real x[NX];
#pragma unroll
  for (int a = 0; a < NX; ++a) x[a] = ra.x0[a];
  __syncthreads();
  for (int t = 0; t < p.T; ++t) {
    Real eps[4], u[NU], pert[NU];
    normals<Real, NU>(p.key0, p.key1, wc, k, 0u, (uint32_t)t, eps);
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      pert[a] = p.noise_std[a] * eps[a];
      u[a] = ra.u_nom[t * NU + a] + pert[a];
    }
    Real cu = 0;
    if constexpr (DYN == kDynQuadHybrid)
      if (p.ctrl_cost) cu = control_cost<Real>(p, ra.u_nom + t * NU, pert);
    Real z[D];
    lwpr_input<DYN>(x, u, z);
    direct_mixture<Real, D>(m, rec, z, tile, out);
    Real acc[NO];
    if (p.M > 0) {
      Real xi[8];
      normals<Real, NO>(p.key0, p.key1, wd, k, mm, (uint32_t)t, xi);
#pragma unroll
      for (int o = 0; o < NO; ++o) acc[o] = out[o] + sqrt_(out[kMaxOut + o]) * xi[o];
    } else {
#pragma unroll
      for (int o = 0; o < NO; ++o) acc[o] = out[o];
    }
    Real xn[NX];
    euler_step<Real>(DYN, p.dt, x, acc, u, xn);
#pragma unroll
    for (int a = 0; a < NX; ++a) x[a] = xn[a];
    const Real c = p.dt * state_cost<Real>(p, obs, x) + cu;
    if (active) ra.cost[s * p.T + t] = c;
  }
}

// Small problems: 16 lanes per sub-rollout split the local models of every
// output (merged by xor shuffles in a fixed order), 16 sub-rollouts per block;
// lane 0 of each sub-rollout samples, steps Euler and writes the cost.  The
// lanes draw the noise of the next 16 steps together (lane l: step t + l), and
// a model that fits in LDS is staged once, so a step has a single barrier.
// Sixteen times the threads of the lane-per-sub-rollout kernel, for grids
// that would otherwise leave most of the chip idle.
constexpr int kGroupLanes = 16, kGroupRows = 16, kGroupChunk = 16;
template <typename Real, int DYN>
__global__ void __launch_bounds__(kGroupLanes *kGroupRows) rollout_group_kernel(RolloutArgs<Real> ra, ModelArgs m,
                                                                              const Real *__restrict__ rec) {
  using DD = DynDims<DYN>;
  constexpr int D = DD::D, NX = DD::NX, NU = DD::NU, NO = DD::NO;
  constexpr int RS = rec_stride<Real, D>(), TM = tile_models<Real, D>();
  __shared__ Real tile[TM * RS];
  __shared__ Real zs[kGroupRows][D];
  // applied controls u_nom + sigma eps and next-state draws of the chunk's steps
  __shared__ Real us_s[kGroupChunk][kGroupRows][4], xi_s[kGroupChunk][kGroupRows][8];
  __shared__ Real obs[kMaxObs * 3];
  const ProbDev<Real> &p = ra.p;
  for (int i = threadIdx.x; i < 3 * p.n_obs; i += blockDim.x) obs[i] = p.obs[i];
  const bool resident = m.Ltot <= TM;   // the whole model in LDS for the whole rollout
  if (resident)
    for (int i = threadIdx.x; i < m.Ltot * RS; i += blockDim.x) tile[i] = rec[i];
  const int g = threadIdx.x / kGroupLanes, l = threadIdx.x % kGroupLanes;
  const int64_t s = (int64_t)blockIdx.x * kGroupRows + g;
  const bool active = s < (int64_t)p.K * p.Ms;
  const uint32_t k = active ? (uint32_t)(s / p.Ms) : 0u, mm = active ? (uint32_t)(s % p.Ms) : 0u;
  const uint32_t it = *ra.iter;
  const uint32_t wc = stream_word(kTagCtrl, p.problem_id, it);
  const uint32_t wd = stream_word(kTagDyn, p.problem_id, it);
  Real x[NX], u[NU];
#pragma unroll
  for (int a = 0; a < NX; ++a) x[a] = ra.x0[a];
  for (int t = 0; t < p.T; ++t) {
    const int tc = t % kGroupChunk;
    if (tc == 0) {
      __syncthreads();   // lane 0 of every row is done with the previous chunk
      if (active && t + l < p.T) {
        Real e[NU], pert[NU];
        normals<Real, NU>(p.key0, p.key1, wc, k, 0u, (uint32_t)(t + l), e);
#pragma unroll
        for (int a = 0; a < NU; ++a) {
          pert[a] = p.noise_std[a] * e[a];
          us_s[l][g][a] = ra.u_nom[(t + l) * NU + a] + pert[a];
        }
        if (p.M > 0) normals<Real, NO>(p.key0, p.key1, wd, k, mm, (uint32_t)(t + l), xi_s[l][g]);
        // the step's control terms ride in the draw slot the hybrid model leaves unused
        if constexpr (DYN == kDynQuadHybrid)
          if (p.ctrl_cost) xi_s[l][g][7] = control_cost<Real>(p, ra.u_nom + (t + l) * NU, pert);
      }
    }
    if (l == 0) {
      Real z[D];
      if (active) {
#pragma unroll
        for (int a = 0; a < NU; ++a) u[a] = us_s[tc][g][a];
        lwpr_input<DYN>(x, u, z);
      } else {
#pragma unroll
        for (int a = 0; a < D; ++a) z[a] = 0;
      }
#pragma unroll
      for (int a = 0; a < D; ++a) zs[g][a] = z[a];
    }
    __syncthreads();
    Real zz[D];
#pragma unroll
    for (int a = 0; a < D; ++a) zz[a] = zs[g][a];
    Real acc[NO];
    for (int o = 0; o < NO; ++o) {
      MixStat<Real> st = mix_empty<Real>();
      for (int j0 = m.L_off[o]; j0 < m.L_off[o + 1]; j0 += TM) {
        const int nj = min(TM, m.L_off[o + 1] - j0);
        const Real *base = tile;
        if (resident) {
          base = tile + (size_t)j0 * RS;
        } else {
          __syncthreads();
          for (int i = threadIdx.x; i < nj * RS; i += blockDim.x) tile[i] = rec[(size_t)j0 * RS + i];
          __syncthreads();
        }
        for (int jj = l; jj < nj; jj += kGroupLanes) {
          Real q, y;
          eval_record<Real, D>(base + jj * RS, zz, q, y);
          mix_add<false>(st, (Real)-0.5 * q, y, base[jj * RS + RS - 1]);
        }
      }
#pragma unroll
      for (int msk = 8; msk >= 1; msk >>= 1) st = mix_merge<false>(st, shfl_stat(st, msk));
      if (l == 0) {   // every lane holds the merged statistics; lane 0 owns the draws
        Real mu, v;
        mix_finish(st, &mu, &v);
        acc[o] = p.M > 0 ? mu + sqrt_(v) * xi_s[tc][g][o] : mu;
      }
    }
    if (l == 0 && active) {
      Real xn[NX];
      euler_step<Real>(DYN, p.dt, x, acc, u, xn);
#pragma unroll
      for (int a = 0; a < NX; ++a) x[a] = xn[a];
      Real c = p.dt * state_cost<Real>(p, obs, x);
      if constexpr (DYN == kDynQuadHybrid)
        if (p.ctrl_cost) c += xi_s[tc][g][7];
      ra.cost[s * p.T + t] = c;
    }
  }
}

template <typename Real>
static hipError_t rollout_group_t(const RolloutArgs<Real> &ra, const ModelArgs &m, const void *rec,
                                  hipStream_t s) {
  const int64_t n = (int64_t)ra.p.K * ra.p.Ms;
  const dim3 grid((unsigned)((n + kGroupRows - 1) / kGroupRows)), block(kGroupLanes * kGroupRows);
  if (ra.p.dyn == kDynPointMass2D)
    hipLaunchKernelGGL((rollout_group_kernel<Real, kDynPointMass2D>), grid, block, 0, s, ra, m, (const Real *)rec);
  else if (ra.p.dyn == kDynQuadHybrid)
    hipLaunchKernelGGL((rollout_group_kernel<Real, kDynQuadHybrid>), grid, block, 0, s, ra, m, (const Real *)rec);
  else
    hipLaunchKernelGGL((rollout_group_kernel<Real, kDynQuad12>), grid, block, 0, s, ra, m, (const Real *)rec);
  return hipGetLastError();
}

template <typename Real>
static hipError_t rollout_direct_t(const RolloutArgs<Real> &ra, const ModelArgs &m, const void *rec,
                                   hipStream_t s) {
  const int64_t n = (int64_t)ra.p.K * ra.p.Ms;
  // fewer sub-rollouts than 32 lanes per compute unit: split the models over lanes
  if (n < 256 * 32) return rollout_group_t(ra, m, rec, s);
  const unsigned nb = (unsigned)((n + 127) / 128);
  if (ra.p.dyn == kDynPointMass2D) {
    constexpr int D = 6;
    const size_t sh = (size_t)(tile_models<Real, D>() * rec_stride<Real, D>() + 128 * 2 * kMaxOut +
                               3 * kMaxObs) * sizeof(Real);
    hipLaunchKernelGGL((rollout_direct_kernel<Real, kDynPointMass2D>), dim3(nb), dim3(128), sh, s,
                       ra, m, (const Real *)rec);
  } else if (ra.p.dyn == kDynQuadHybrid) {
    constexpr int D = 4;
    const size_t sh = (size_t)(tile_models<Real, D>() * rec_stride<Real, D>() + 128 * 2 * kMaxOut +
                               3 * kMaxObs) * sizeof(Real);
    hipLaunchKernelGGL((rollout_direct_kernel<Real, kDynQuadHybrid>), dim3(nb), dim3(128), sh, s,
                       ra, m, (const Real *)rec);
  } else {
    constexpr int D = 16;
    const size_t sh = (size_t)(tile_models<Real, D>() * rec_stride<Real, D>() + 128 * 2 * kMaxOut +
                               3 * kMaxObs) * sizeof(Real);
    hipLaunchKernelGGL((rollout_direct_kernel<Real, kDynQuad12>), dim3(nb), dim3(128), sh, s, ra, m,
                       (const Real *)rec);
  }
  return hipGetLastError();
}

hipError_t launch_rollout_direct(int dtype, const void *rargs, const ModelArgs &m, const void *rec,
                                 hipStream_t s) {
  return dtype == PI_F64 ? rollout_direct_t<double>(*(const RolloutArgs<double> *)rargs, m, rec, s)
                         : rollout_direct_t<float>(*(const RolloutArgs<float> *)rargs, m, rec, s);
}

// -------------------------------------------------- sub-rollout average
// cbar_{k,t} = (1/M) sum_m c_{k,m,t} (Sec. 3.2), summed in order of m.
template <typename Real>
__global__ void subcost_reduce_kernel(const Real *__restrict__ sub, Real *__restrict__ cost, int K,
                                      int Ms, int T) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)K * T) return;
  const int64_t k = i / T, t = i % T;
  Real acc = 0;
  for (int mm = 0; mm < Ms; ++mm) acc += sub[(k * Ms + mm) * T + t];
  cost[i] = acc / (Real)Ms;
}

hipError_t launch_subcost_reduce(int dtype, const void *sub, void *cost, int K, int Ms, int T,
                                 hipStream_t s) {
  const int64_t n = (int64_t)K * T;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (dtype == PI_F64)
    hipLaunchKernelGGL(subcost_reduce_kernel<double>, dim3(nb), dim3(256), 0, s,
                       (const double *)sub, (double *)cost, K, Ms, T);
  else
    hipLaunchKernelGGL(subcost_reduce_kernel<float>, dim3(nb), dim3(256), 0, s, (const float *)sub,
                       (float *)cost, K, Ms, T);
  return hipGetLastError();
}

// ------------------------------------------------------------- update
// Eq. (2) with the cost-to-go of Sec. 3.1.  Three stages, all in double:
//  (1) one lane per rollout k: suffix sums S[i][k] = sum_{t>=i} cost[k][t];
//  (2) block (chunk c, step i): over its rollouts, the local minimum m_c,
//      Z_c = sum exp(-(S - m_c)/lambda) and N_c = sum exp(...) eps_{k,i};
//  (3) one lane per step i merges the chunks in order (log-sum-exp shifts)
//      and applies u_i += N / Z.  An optional stage (4) writes P_{k,i}.
constexpr int kUpdChunk = 2048;   // rollouts per stage-2 block
constexpr int kUpdThreads = 256;

size_t update_ws_bytes(int K, int T) {
  const int C = (K + kUpdChunk - 1) / kUpdChunk;
  return align_up((size_t)K * T * 8, 256) + align_up((size_t)T * C * (2 + kMaxU) * 8, 256) +
         align_up((size_t)T * 2 * 8, 256);
}

// Suffix sums S[t][k] = sum_{t' >= t} cost[k][t'] in double.  A block holds 64
// rollouts and splits the horizon into 4 segments, one wave each: every lane
// sums its (rollout, segment), the segment totals meet in LDS, and each lane
// walks its segment backwards from the total of the later segments; the S
// stores of a wave cover 64 consecutive rollouts.  Two ways to read the costs:
// each lane straight along its own row (every load of a wave touches 64 rows,
// but all of a lane's loads are in flight at once: best when the grid is
// small), or through a per-wave LDS tile in chunks of 16 steps (each load
// covers 16 consecutive steps of 4 rollouts: best when bandwidth matters).
constexpr int kSufK = 64, kSufSeg = 4, kSufChunk = 16;
template <typename Real, bool kStaged>
__global__ void __launch_bounds__(kSufK * kSufSeg) suffix_kernel(const Real *__restrict__ cost, int K, int T,
                                                                 double *__restrict__ S) {
  __shared__ double tile[kStaged ? kSufSeg : 1][kSufK][kSufChunk + 1];
  __shared__ double tot[kSufSeg][kSufK];
  const int lane = threadIdx.x % kSufK, seg = threadIdx.x / kSufK;
  const int k0 = blockIdx.x * kSufK, k = k0 + lane;
  const int lo = (int)((int64_t)seg * T / kSufSeg), hi = (int)((int64_t)(seg + 1) * T / kSufSeg);
  const Real *row = cost + (int64_t)min(k, K - 1) * T;
  double (*tl)[kSufChunk + 1] = tile[kStaged ? seg : 0];
  // chunk [c0, c0 + w) of the segment into this wave's tile (rows past K read row K-1)
  auto load = [&](int c0, int w) {
    for (int e = lane; e < kSufK * kSufChunk; e += kSufK) {
      const int r = e / kSufChunk, c = e % kSufChunk;
      if (c < w) tl[r][c] = (double)cost[(int64_t)min(k0 + r, K - 1) * T + c0 + c];
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  };
  double sum = 0.0;
  if constexpr (kStaged) {
    for (int c0 = lo; c0 < hi; c0 += kSufChunk) {
      const int w = min(kSufChunk, hi - c0);
      load(c0, w);
      for (int c = 0; c < w; ++c) sum += tl[lane][c];
      __builtin_amdgcn_wave_barrier();
    }
  } else {
    for (int t = lo; t < hi; ++t) sum += (double)row[t];
  }
  tot[seg][lane] = sum;
  __syncthreads();
  double acc = 0.0;
  for (int j = kSufSeg - 1; j > seg; --j) acc += tot[j][lane];
  if constexpr (kStaged) {
    for (int c1 = hi; c1 > lo; c1 -= kSufChunk) {
      const int c0 = max(lo, c1 - kSufChunk), w = c1 - c0;
      load(c0, w);
      for (int c = w - 1; c >= 0; --c) {
        acc += tl[lane][c];
        if (k < K) S[(int64_t)(c0 + c) * K + k] = acc;
      }
      __builtin_amdgcn_wave_barrier();
    }
  } else {
    if (k >= K) return;
    for (int t = hi - 1; t >= lo; --t) {
      acc += (double)row[t];
      S[(int64_t)t * K + k] = acc;
    }
  }
}

template <typename Real>
__global__ void __launch_bounds__(kUpdThreads) update_chunk_kernel(ProbDev<Real> p, double lambda,
                                                                   int weighting,
                                                                   const uint32_t *__restrict__ iter,
                                                                   const double *__restrict__ S,
                                                                   double *__restrict__ part) {
  __shared__ double red[kUpdThreads];
  __shared__ double acc[kUpdThreads][kMaxU + 1];
  const int c = blockIdx.x, i = blockIdx.y, C = gridDim.x;
  const int K = p.K;
  const int k0 = c * kUpdChunk, k1 = min(K, k0 + kUpdChunk);
  const double *Si = S + (int64_t)(weighting == PI_W_TRAJECTORY ? 0 : i) * K;
  double mn = 1.0 / 0.0;
  for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) mn = fmin(mn, Si[k]);
  red[threadIdx.x] = mn;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  mn = red[0];
  const uint32_t wc = stream_word(kTagCtrl, p.problem_id, *iter);
  double z = 0.0, n[kMaxU] = {0.0, 0.0, 0.0, 0.0};
  for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    const double om = exp(-(Si[k] - mn) / lambda);
    Real eps[4];
    normals<Real, 4>(p.key0, p.key1, wc, (uint32_t)k, 0u, (uint32_t)i, eps);
    z += om;
#pragma unroll
    for (int a = 0; a < kMaxU; ++a)
      if (a < p.n_u) n[a] += om * (double)(p.noise_std[a] * eps[a]);
  }
  acc[threadIdx.x][0] = z;
#pragma unroll
  for (int a = 0; a < kMaxU; ++a) acc[threadIdx.x][1 + a] = n[a];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q <= kMaxU; ++q) acc[threadIdx.x][q] += acc[threadIdx.x + w][q];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double *o = part + ((int64_t)i * C + c) * (2 + kMaxU);
    o[0] = mn;
    for (int q = 0; q <= kMaxU; ++q) o[1 + q] = acc[0][q];
  }
}

template <typename Real>
__global__ void update_apply_kernel(int T, int C, int n_u, double lambda,
                                    const double *__restrict__ part,
                                    Real *__restrict__ u_nom, double *__restrict__ norm,
                                    uint32_t *__restrict__ iter) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  // the iteration's draws have all been consumed: advance the iteration word
  if (i == 0) *iter += 1u;
  if (i >= T) return;
  const double *pi_ = part + (int64_t)i * C * (2 + kMaxU);
  double mn = 1.0 / 0.0;
  for (int c = 0; c < C; ++c) mn = fmin(mn, pi_[c * (2 + kMaxU)]);
  double z = 0.0, n[kMaxU] = {0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < C; ++c) {
    const double *q = pi_ + c * (2 + kMaxU);
    const double f = (q[0] == mn) ? 1.0 : exp(-(q[0] - mn) / lambda);
    z += q[1] * f;
    for (int a = 0; a < kMaxU; ++a) n[a] += q[2 + a] * f;
  }
  for (int a = 0; a < n_u; ++a) u_nom[i * n_u + a] = (Real)((double)u_nom[i * n_u + a] + n[a] / z);
  norm[2 * i] = mn;
  norm[2 * i + 1] = z;
}

__global__ void update_weights_kernel(int K, int T, double lambda, int weighting,
                                      const double *__restrict__ S, const double *__restrict__ norm,
                                      double *__restrict__ W) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)K * T) return;
  const int64_t i = idx / K, k = idx % K;
  const double s = S[(weighting == PI_W_TRAJECTORY ? 0 : i) * (int64_t)K + k];
  W[idx] = exp(-(s - norm[2 * i]) / lambda) / norm[2 * i + 1];
}

template <typename Real>
static hipError_t update_t(const ProbDev<Real> &p, const Real *cost, const uint32_t *iter,
                           Real *u_nom, double *W, void *ws, double lambda, int weighting,
                           hipStream_t s) {
  const int K = p.K, T = p.T, C = (K + kUpdChunk - 1) / kUpdChunk;
  double *S = (double *)ws;
  double *part = (double *)((char *)ws + align_up((size_t)K * T * 8, 256));
  double *norm = (double *)((char *)part + align_up((size_t)T * C * (2 + kMaxU) * 8, 256));
  const unsigned nsb = (unsigned)((K + kSufK - 1) / kSufK);
  if (nsb >= 256)   // enough blocks to cover the compute units: read through LDS
    hipLaunchKernelGGL((suffix_kernel<Real, true>), dim3(nsb), dim3(kSufK * kSufSeg), 0, s, cost, K, T, S);
  else
    hipLaunchKernelGGL((suffix_kernel<Real, false>), dim3(nsb), dim3(kSufK * kSufSeg), 0, s, cost, K, T, S);
  hipLaunchKernelGGL(update_chunk_kernel<Real>, dim3(C, T), dim3(kUpdThreads), 0, s, p, lambda,
                     weighting, iter, (const double *)S, part);
  hipLaunchKernelGGL(update_apply_kernel<Real>, dim3((T + 63) / 64), dim3(64), 0, s, T, C, p.n_u,
                     lambda, (const double *)part, u_nom, norm, const_cast<uint32_t *>(iter));
  if (W) {
    const int64_t n = (int64_t)K * T;
    hipLaunchKernelGGL(update_weights_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, K,
                       T, lambda, weighting, (const double *)S, (const double *)norm, W);
  }
  return hipGetLastError();
}

hipError_t launch_update(int dtype, const void *pargs, const void *cost, const uint32_t *iter,
                         void *u_nom, double *weights, void *ws, int, double lambda, int weighting,
                         hipStream_t s) {
  if (dtype == PI_F64)
    return update_t<double>(*(const ProbDev<double> *)pargs, (const double *)cost, iter,
                            (double *)u_nom, weights, ws, lambda, weighting, s);
  return update_t<float>(*(const ProbDev<float> *)pargs, (const float *)cost, iter, (float *)u_nom,
                         weights, ws, lambda, weighting, s);
}

// ------------------------------------------------------------ RH shift
// The plant step executes u_nom[0] under the PLANT stream.  Kernel 1: block
// (o, c) evaluates 64 local models of output o at z = [x0 ; u_nom[0]], one per
// lane, and merges them into one partial statistic (fixed tree order).
// Kernel 2 (one block): merges the partials of every output in order, samples
// the accelerations, steps Euler and shifts the plan left by one step (last
// control repeated).  The iteration word is read, not advanced.
constexpr int kShiftThreads = 64;

size_t shift_partial_bytes(const ModelArgs &m, int dtype) {
  int Lmax = 1;
  for (int o = 0; o < m.n_out; ++o) Lmax = max(Lmax, m.L_off[o + 1] - m.L_off[o]);
  const int C = (Lmax + kShiftThreads - 1) / kShiftThreads;
  return align_up((size_t)m.n_out * C * 5 * (dtype == PI_F64 ? 8 : 4), 256);
}

template <typename Real, int DYN>
__global__ void __launch_bounds__(kShiftThreads) plant_partial_kernel(ModelArgs m,
                                                                      const Real *__restrict__ rec,
                                                                      const Real *__restrict__ x0,
                                                                      const Real *__restrict__ u_nom,
                                                                      MixStat<Real> *__restrict__ part) {
  using DD = DynDims<DYN>;
  constexpr int D = DD::D, NX = DD::NX, NU = DD::NU;
  constexpr int RS = rec_stride<Real, D>();
  __shared__ MixStat<Real> red[kShiftThreads];
  const int o = blockIdx.y, c = blockIdx.x, C = gridDim.x;
  Real z[D], x[NX], u[NU];
#pragma unroll
  for (int a = 0; a < NX; ++a) x[a] = x0[a];
#pragma unroll
  for (int a = 0; a < NU; ++a) u[a] = u_nom[a];
  lwpr_input<DYN>(x, u, z);
  MixStat<Real> st = mix_empty<Real>();
  const int j = m.L_off[o] + c * kShiftThreads + threadIdx.x;
  if (j < m.L_off[o + 1]) {
    Real q, y;
    eval_record<Real, D>(rec + (size_t)j * RS, z, q, y);
    mix_add<false>(st, (Real)-0.5 * q, y, rec[(size_t)j * RS + RS - 1]);
  }
  red[threadIdx.x] = st;
  __syncthreads();
  for (int w = kShiftThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = mix_merge<false>(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[o * C + c] = red[0];
}

template <typename Real, int DYN>
__global__ void __launch_bounds__(256) plant_apply_kernel(ProbDev<Real> p, int C,
                                                          const MixStat<Real> *__restrict__ part,
                                                          Real *__restrict__ x0, Real *__restrict__ u_nom,
                                                          const uint32_t *__restrict__ iter) {
  using DD = DynDims<DYN>;
  constexpr int NX = DD::NX, NU = DD::NU, NO = DD::NO;
  __shared__ Real xnew[kMaxX];
  if (threadIdx.x == 0) {
    const uint32_t it = *iter;
    Real xi[8], acc[NO], xs[NX], xn[NX];
    normals<Real, NO>(p.key0, p.key1, stream_word(kTagPlant, p.problem_id, it), 0u, 0u, 0u, xi);
    for (int o = 0; o < NO; ++o) {
      MixStat<Real> st = part[o * C];
      for (int c = 1; c < C; ++c) st = mix_merge<false>(st, part[o * C + c]);
      Real mu, v;
      mix_finish(st, &mu, &v);
      acc[o] = mu + sqrt_(v) * xi[o];
    }
    Real u0[NU];
    for (int a = 0; a < NX; ++a) xs[a] = x0[a];
    for (int a = 0; a < NU; ++a) u0[a] = u_nom[a];
    euler_step<Real>(DYN, p.dt, xs, acc, u0, xn);
    for (int a = 0; a < NX; ++a) xnew[a] = xn[a];
  }
  __syncthreads();
  // Shift left by one control in place.  Chunk by chunk every lane reads its
  // new value before any lane writes; a chunk only reads indices at or above
  // its own start, which no earlier chunk has written.
  const int n = p.T * NU;
  for (int base = 0; base < n; base += blockDim.x) {
    const int i = base + threadIdx.x;
    Real v = 0;
    if (i < n) v = (i + NU < n) ? u_nom[i + NU] : u_nom[i];
    __syncthreads();
    if (i < n) u_nom[i] = v;
    __syncthreads();
  }
  if (threadIdx.x < NX) x0[threadIdx.x] = xnew[threadIdx.x];
}

template <typename Real>
static hipError_t rh_shift_t(const ProbDev<Real> &p, const ModelArgs &m, const void *rec, void *part,
                             void *x0, void *u_nom, const uint32_t *iter, hipStream_t s) {
  int Lmax = 1;
  for (int o = 0; o < m.n_out; ++o) Lmax = max(Lmax, m.L_off[o + 1] - m.L_off[o]);
  const int C = (Lmax + kShiftThreads - 1) / kShiftThreads;
  const dim3 grid(C, m.n_out);
  if (p.dyn == kDynPointMass2D) {
    hipLaunchKernelGGL((plant_partial_kernel<Real, kDynPointMass2D>), grid, dim3(kShiftThreads), 0, s, m,
                       (const Real *)rec, (const Real *)x0, (const Real *)u_nom, (MixStat<Real> *)part);
    hipLaunchKernelGGL((plant_apply_kernel<Real, kDynPointMass2D>), dim3(1), dim3(256), 0, s, p, C,
                       (const MixStat<Real> *)part, (Real *)x0, (Real *)u_nom, iter);
  } else if (p.dyn == kDynQuadHybrid) {
    hipLaunchKernelGGL((plant_partial_kernel<Real, kDynQuadHybrid>), grid, dim3(kShiftThreads), 0, s, m,
                       (const Real *)rec, (const Real *)x0, (const Real *)u_nom, (MixStat<Real> *)part);
    hipLaunchKernelGGL((plant_apply_kernel<Real, kDynQuadHybrid>), dim3(1), dim3(256), 0, s, p, C,
                       (const MixStat<Real> *)part, (Real *)x0, (Real *)u_nom, iter);
  } else {
    hipLaunchKernelGGL((plant_partial_kernel<Real, kDynQuad12>), grid, dim3(kShiftThreads), 0, s, m,
                       (const Real *)rec, (const Real *)x0, (const Real *)u_nom, (MixStat<Real> *)part);
    hipLaunchKernelGGL((plant_apply_kernel<Real, kDynQuad12>), dim3(1), dim3(256), 0, s, p, C,
                       (const MixStat<Real> *)part, (Real *)x0, (Real *)u_nom, iter);
  }
  return hipGetLastError();
}

hipError_t launch_rh_shift(int dtype, const void *pargs, const ModelArgs &m, const void *rec,
                           void *part, void *x0, void *u_nom, const uint32_t *iter, hipStream_t s) {
  return dtype == PI_F64
             ? rh_shift_t<double>(*(const ProbDev<double> *)pargs, m, rec, part, x0, u_nom, iter, s)
             : rh_shift_t<float>(*(const ProbDev<float> *)pargs, m, rec, part, x0, u_nom, iter, s);
}

// Clears one counter with a kernel (graph-capture friendly, no memset node).
__global__ void zero_int_kernel(int *p) { *p = 0; }
__global__ void zero_u32_kernel(uint32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}
hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)nb), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
hipError_t launch_zero_int(int *p, hipStream_t s) {
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, p);
  return hipGetLastError();
}

// ------------------------------------------------------ stream access
__global__ void philox_kernel(const uint32_t *__restrict__ ctr, uint32_t k0, uint32_t k1,
                              uint32_t *__restrict__ out, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const Philox4 r = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
  for (int q = 0; q < 4; ++q) out[4 * i + q] = r.v[q];
}

hipError_t launch_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out, int64_t N,
                         hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, ctr, k0, k1,
                     out, N);
  return hipGetLastError();
}

// One lane per (k, t): the same normals<> calls as the rollout, update and
// shift kernels.
template <typename Real>
__global__ void noise_kernel(ProbDev<Real> p, int tag, const uint32_t *__restrict__ iter, int k0,
                             int nk, int m, Real *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t word = stream_word((uint32_t)tag, p.problem_id, *iter);
  Real v[8];
  if (tag == kTagPlant) {
    if (i != 0) return;
    normals_n<Real>(p.n_out, p.key0, p.key1, word, 0u, 0u, 0u, v);
    for (int o = 0; o < p.n_out; ++o) out[o] = v[o];
    return;
  }
  if (i >= (int64_t)nk * p.T) return;
  const uint32_t k = (uint32_t)(k0 + i / p.T), t = (uint32_t)(i % p.T);
  if (tag == kTagCtrl) {
    normals_n<Real>(p.n_u, p.key0, p.key1, word, k, 0u, t, v);
    for (int a = 0; a < p.n_u; ++a) out[i * p.n_u + a] = p.noise_std[a] * v[a];
  } else {
    normals_n<Real>(p.n_out, p.key0, p.key1, word, k, (uint32_t)m, t, v);
    for (int o = 0; o < p.n_out; ++o) out[i * p.n_out + o] = v[o];
  }
}

hipError_t launch_noise(int dtype, const void *pargs, int tag, const uint32_t *iter, int k0, int nk,
                        int m, void *out, hipStream_t s) {
  const int T = dtype == PI_F64 ? ((const ProbDev<double> *)pargs)->T : ((const ProbDev<float> *)pargs)->T;
  const int64_t n = tag == kTagPlant ? 1 : (int64_t)nk * T;
  if (n == 0) return hipSuccess;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (dtype == PI_F64)
    hipLaunchKernelGGL(noise_kernel<double>, dim3(nb), dim3(256), 0, s,
                       *(const ProbDev<double> *)pargs, tag, iter, k0, nk, m, (double *)out);
  else
    hipLaunchKernelGGL(noise_kernel<float>, dim3(nb), dim3(256), 0, s, *(const ProbDev<float> *)pargs,
                       tag, iter, k0, nk, m, (float *)out);
  return hipGetLastError();
}

}  // namespace pi2rh
