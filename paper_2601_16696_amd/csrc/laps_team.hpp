// Register-tile helpers shared by the per-chain kernels: a team of T lanes
// holds one chain; lane r owns octs r + q T (eight consecutive coordinates,
// one Philox block each) of a row of stride ld.
#pragma once
#include "laps_internal.hpp"

namespace laps {

template <class Real, int Q>
struct Tile {
  Real v[Q][8];
};

template <class Real>
__device__ __forceinline__ void ld8(const Real *p, Real (&v)[8]);
template <>
__device__ __forceinline__ void ld8<float>(const float *p, float (&v)[8]) {
  const float4 a = *reinterpret_cast<const float4 *>(p);
  const float4 b = *reinterpret_cast<const float4 *>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
template <>
__device__ __forceinline__ void ld8<double>(const double *p, double (&v)[8]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double2 a = *reinterpret_cast<const double2 *>(p + 2 * k);
    v[2 * k] = a.x;
    v[2 * k + 1] = a.y;
  }
}
template <class Real>
__device__ __forceinline__ void st8(Real *p, const Real (&v)[8]);
template <>
__device__ __forceinline__ void st8<float>(float *p, const float (&v)[8]) {
  *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
  *reinterpret_cast<float4 *>(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
}
template <>
__device__ __forceinline__ void st8<double>(double *p, const double (&v)[8]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) *reinterpret_cast<double2 *>(p + 2 * k) = make_double2(v[2 * k], v[2 * k + 1]);
}

// Loads the lane's octs of one row; coordinates >= d read as zero.
template <class Real, int Q>
__device__ __forceinline__ void load_row(const Real *row, int r, int T, int64_t d, bool act, Real (&v)[Q][8]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t e0 = 8 * (int64_t)(r + q * T);
    if (act && e0 < d) {
      ld8<Real>(row + e0, v[q]);
      if (e0 + 8 > d) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (e0 + i >= d) v[q][i] = Real(0);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[q][i] = Real(0);
    }
  }
}

template <class Real, int Q>
__device__ __forceinline__ void store_row(Real *row, int r, int T, int64_t d, const Real (&v)[Q][8]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t e0 = 8 * (int64_t)(r + q * T);
    if (e0 < d) st8<Real>(row + e0, v[q]);
  }
}

// Standard normals for the lane's octs (zero beyond d).
template <class Real, int Q>
__device__ __forceinline__ void lane_normals(uint64_t seed, uint64_t m, int r, int T, int64_t d, uint64_t t,
                                             uint32_t tag, uint32_t sub, Real (&z)[Q][8]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t oct = r + q * T;
    if (8 * oct < d) {
      normals8<Real>(seed, m, (uint64_t)oct, t, tag, sub, z[q]);
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (8 * oct + i >= d) z[q][i] = Real(0);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) z[q][i] = Real(0);
    }
  }
}

// Standard normals of one oct (zero beyond d), generated where they are
// consumed so that no [Q][8] array of them stays live.
template <class Real>
__device__ __forceinline__ void oct_normals(uint64_t seed, uint64_t m, int64_t oct, int64_t d, uint64_t t,
                                            uint32_t tag, uint32_t sub, Real (&z)[8]) {
  if (8 * oct < d) {
    normals8<Real>(seed, m, (uint64_t)oct, t, tag, sub, z);
    if (8 * oct + 8 > d) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (8 * oct + i >= d) z[i] = Real(0);
    }
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = Real(0);
  }
}

// Per-dimension sums over every chain this workgroup visited, written as one
// partial row per workgroup: teams inside a wavefront are combined by xor
// butterflies, wavefronts in a fixed order through LDS.
template <class Real, int Q>
__device__ __forceinline__ void write_partials(double *partials, int64_t d, int64_t ld, double (&S)[4][Q][8],
                                               double *buf, int T, int r) {
  double *P = partials + (size_t)blockIdx.x * 4 * ld;
  if ((int)blockDim.x == T) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int64_t e0 = 8 * (int64_t)(r + q * T);
        if (e0 < d)
#pragma unroll
          for (int i = 0; i < 8; ++i) P[k * ld + e0 + i] = S[k][q][i];
      }
    return;
  }
  // T < blockDim: first fold teams that share a wavefront (xor butterflies;
  // the levels of 16 and 32 lanes by lane swaps; in mode 2 the level of 32 is
  // left to the reader, which adds the two halves first, as that level would)
  const int mode = partials_mode(blockDim.x, T, Q);
  for (int msk = T; msk < 16; msk <<= 1) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) S[k][q][i] += __shfl_xor(S[k][q][i], msk);
  }
  if (T <= 16) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) S[k][q][i] = xor_pair_sum<16>(S[k][q][i]);
  }
  if (T <= 32 && mode != 2) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) S[k][q][i] = xor_pair_sum<32>(S[k][q][i]);
  }
  // then wavefront (or multi-wave team) groups in order, accumulated in LDS
  const int lanes = T;  // lanes holding a distinct set of dims
  const int groups = blockDim.x / (T < 64 ? 64 : T);
  const int grp = threadIdx.x / (T < 64 ? 64 : T);
  const int lig = threadIdx.x - grp * (T < 64 ? 64 : T);  // lane index inside its group
  const int span = 8 * Q * lanes;
  if (mode == 2) {
    // half hg of wavefront grp stages its rows as group 2 grp + hg (its lane
    // index lh is the team lane: after the folds below 32 lanes its first T
    // lanes hold the half's sums); the reader adds half 0 + half 1 of each
    // wavefront, then the wavefronts in order from 0
    const int hg = (threadIdx.x >> 5) & 1, lh = threadIdx.x & 31;
    __syncthreads();  // the buffer may hold other teams' staged rows until here
    if (lh < lanes) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int i = 0; i < 8; ++i)
            buf[((2 * grp + hg) * 4 + k) * span + (q * lanes + lh) * 8 + i] = S[k][q][i];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 4 * span; e += blockDim.x) {
      const int k = e / span, c = e - k * span;
      double v = 0.0;
      for (int gI = 0; gI < groups; ++gI)
        v += buf[((2 * gI) * 4 + k) * span + c] + buf[((2 * gI + 1) * 4 + k) * span + c];
      if (8 * (c / 8) < d) P[k * ld + c] = v;
    }
    return;
  }
  if (mode == 1) {
    // every group stages its rows at once (after a barrier: the buffer may
    // hold other teams' staged rows until then), one barrier, then the
    // workgroup's threads add the groups in order (0 + group 0 + group 1 + ...,
    // the order of the loop below); element c of a row is coordinate c of the
    // chain (c = 8 (q T + lane) + i)
    __syncthreads();
    if (lig < lanes) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int i = 0; i < 8; ++i) buf[(grp * 4 + k) * span + (q * lanes + lig) * 8 + i] = S[k][q][i];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 4 * span; e += blockDim.x) {
      const int k = e / span, c = e - k * span;
      double v = 0.0;
      for (int gI = 0; gI < groups; ++gI) v += buf[(gI * 4 + k) * span + c];
      if (8 * (c / 8) < d) P[k * ld + c] = v;
    }
    return;
  }
  for (int gI = 0; gI < groups; ++gI) {
    if (grp == gI && lig < lanes) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int idx = k * span + (q * lanes + lig) * 8 + i;
            buf[idx] = (gI == 0 ? 0.0 : buf[idx]) + S[k][q][i];
          }
    }
    __syncthreads();
  }
  if (grp == 0 && lig < lanes) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int64_t e0 = 8 * (int64_t)(r + q * T);
        if (e0 < d)
#pragma unroll
          for (int i = 0; i < 8; ++i) P[k * ld + e0 + i] = buf[k * span + (q * lanes + lig) * 8 + i];
      }
  }
}

template <class Real, int Q>
__device__ __forceinline__ void accumulate_stats(double (&S)[4][Q][8], const double (&K)[Q][8],
                                                 const Real (&x)[Q][8], const Real (&g)[Q][8]) {
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double dx = (double)x[q][i] - K[q][i];
      const double gv = (double)g[q][i];
      S[0][q][i] += dx;
      S[1][q][i] += dx * dx;
      S[2][q][i] += dx * gv;
      S[3][q][i] += gv;
    }
}

template <int Q>
__device__ __forceinline__ void load_shift(const double *K, int r, int T, int64_t d, double (&v)[Q][8]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t e0 = 8 * (int64_t)(r + q * T);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[q][i] = (e0 + i < d) ? K[e0 + i] : 0.0;
  }
}

}  // namespace laps
