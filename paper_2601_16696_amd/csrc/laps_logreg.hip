// Bayesian logistic regression target of the LAPS hot path.
//
// Gradient: for chain positions theta (rows of x), z = X theta over the n data
// rows, r = y - sigmoid(z), grad log p = X^T r - theta and
// log p = sum_n [y z - softplus(z)] - |theta|^2 / 2.
//
// Mixed precision (LAPS_MIXED_BF16): both contractions run on bf16 matrix
// cores (v_mfma_f32_16x16x32_bf16) with float accumulation, fused so z never
// leaves registers: a wavefront holds 16 chains; per 32-row block of X it
// computes z^T (rows x chains) with theta split into bf16 hi + lo parts (X is
// exactly bf16 by construction, so z carries ~2^-17 relative error), applies
// the sigmoid/softplus epilogue in float (log p terms summed in double), and
// accumulates G^T += X^T r^T from the epilogue registers directly: the K
// index of the second product is permuted to the first product's output
// layout, and both operands of X are pre-packed in fragment order.  The n
// rows are split over S workgroup columns; per-split partial sums are
// combined by the per-chain update kernels.
//
// Plain FP64 (LAPS_F64): the same partial-sum interface with a double-precision
// vector-ALU gradient (the baseline the mixed path is measured against).
//
// The per-chain update kernels also serve caller-supplied targets: the
// caller's gradient callback writes one "split" of partial sums (g and log p
// without the prior), and the kernels run unchanged with prior = 0.
#include "laps_team.hpp"

namespace laps {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

void logreg_splits(int64_t n, int64_t N, int prec, int64_t d, int wgs, int &S, int &NB, int &bps) {
  (void)d;
  NB = (int)((n + 31) / 32);
  // chain tiles of one gradient launch: 128 chains per bf16 workgroup (one per
  // CU), 64 per FP64 one (two per CU)
  const int64_t groups = prec != 0 ? (N + 127) / 128 : (N + 63) / 64;
  int64_t target = prec != 0 ? 256 : 512;
  if (wgs > 0) target = wgs;
  int64_t want = target / (groups > 0 ? groups : 1);
  if (want < 1) want = 1;
  if (want > NB) want = NB;
  bps = (int)((NB + want - 1) / want);
  S = (NB + bps - 1) / bps;
}

// The gate's phase word is read at launch but tested only once the launch's
// first independent loads are issued (before its first store), so that its
// latency overlaps theirs; a launch gated off waits for those loads and ends.
__device__ __forceinline__ bool lr_gate(const LogregArgs &a) {
  if (a.gate == 0) return true;
  const DevHyper *H = a.hyp;
  if (a.gate == 1) return H->phase == PH_UNADJ;
  return H->phase == PH_ADJ && H->t < a.max_total;
}

// ---------------------------------------------------------------------------
// operand packing (bf16 paths), once per context
//   Xf[b][h][kc][lane][j] = X[32b + 16h + lane%16][32kc + 16(j/4) + 4(lane/16) + j%4]
//   Xb[b][dc][lane][j]    = X[32b + 16(j/4) + 4(lane/16) + j%4][16dc + lane%16]
//   yf[row]               = y[row] - 1/2 (0 beyond n)
// ---------------------------------------------------------------------------
__global__ void k_lr_pack(const unsigned short *X, const double *y, int64_t n, int64_t d, int64_t ld, int KC,
                          int NB, unsigned short *Xf, unsigned short *Xb, float *yf, double *wy) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nf = (int64_t)NB * 2 * KC * 64;
  if (tid < nf) {
    const int lane = (int)(tid % 64);
    const int64_t rest = tid / 64;
    const int kc = (int)(rest % KC);
    const int h = (int)((rest / KC) % 2);
    const int64_t b = rest / (2 * KC);
    const int64_t row = 32 * b + 16 * h + (lane & 15);
    for (int j = 0; j < 8; ++j) {
      const int64_t col = 32 * kc + 16 * (j >> 2) + 4 * (lane >> 4) + (j & 3);
      Xf[tid * 8 + j] = (row < n && col < d) ? X[row * d + col] : (unsigned short)0;
    }
    return;
  }
  const int64_t t2 = tid - nf;
  const int64_t nbk = (int64_t)NB * 2 * KC * 64;
  if (t2 < nbk) {
    const int lane = (int)(t2 % 64);
    const int64_t rest = t2 / 64;
    const int dc = (int)(rest % (2 * KC));
    const int64_t b = rest / (2 * KC);
    const int64_t col = 16 * dc + (lane & 15);
    for (int j = 0; j < 8; ++j) {
      const int64_t row = 32 * b + 16 * (j >> 2) + 4 * (lane >> 4) + (j & 3);
      Xb[t2 * 8 + j] = (row < n && col < d) ? X[row * d + col] : (unsigned short)0;
    }
    return;
  }
  const int64_t t3 = t2 - nbk;
  if (t3 < (int64_t)NB * 32) {
    yf[t3] = t3 < n ? (float)(y[t3] - 0.5) : 0.0f;
    return;
  }
  // wy[i] = sum_n X_ni (y_n - 1/2) in FP64, rows in order (zero for i >= d)
  const int64_t i = t3 - (int64_t)NB * 32;
  if (i < ld) {
    double acc = 0.0;
    if (i < d)
      for (int64_t r = 0; r < n; ++r)
        acc += (double)__uint_as_float((unsigned)X[r * d + i] << 16) * (y[r] - 0.5);
    wy[i] = acc;
  }
}

// ---------------------------------------------------------------------------
// bf16 matrix-core gradient (d <= 128).  grid (ceil(N/128), S), 512 threads =
// 8 wavefronts, one workgroup per CU: wavefront w owns the 32 chains of pair
// group w % 4 (two 16-chain MFMA tiles, g = 0, 1) and row half w / 4 of the
// split's 32-row blocks (half 0 takes even blocks, half 1 odd ones), so each
// X fragment read from LDS feeds both chain tiles.
//
// Software pipeline.  Iteration it uses the blocks staged for it (its
// epilogue and backward product) and for it + 1 (the forward product of the
// wavefront's next block), while the blocks of it + 2 travel from global
// memory straight into LDS (global_load_lds_dwordx4: one wavefront
// instruction writes 64 consecutive 16-byte fragments).  Three LDS buffers
// rotate as separate arrays with the rotation unrolled, so that the compiler
// can see that a DMA into one buffer does not alias reads of the others and
// waits for it only at the iteration's barrier.  Within an iteration the
// forward products of the next block are independent of the current block's
// sigmoid/softplus epilogue, so the matrix cores and the vector ALU of a
// wavefront work at the same time.  theta's hi and lo products accumulate
// into one register tile.
//
// The products carry z' = z log2(e) (theta is scaled before its hi/lo
// split), so e^{-|z|} is one base-2 exponential.  With the packed label
// ym = y - 1/2 and s = 1/(1 + e^{-|z|}):
//   r = y - sigmoid(z) = ym - copysign(s - 1/2, z')   (s - 1/2 is exact),
//   y z - softplus(z) = ym z - |z|/2 - log(1 + e^{-|z|}).
// The kernel sums only the last two terms per chain (|z'| added, the factors
// 1 + e^{-|z|} in (1, 2] multiplied, one log2 per block); sum_n ym_n z_n =
// theta . (X^T ym) is linear in theta and is added in FP64 by the update
// kernels from the precomputed X^T ym.  Rows past n have X = 0 and ym = 0, so
// they give r = 0 and |z| = 0 and a factor of exactly 2 each, whose log2 (1
// per row) is subtracted.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ void lds_dma16(const bf16x8 *src, bf16x8 *lds_dst) {
  __builtin_amdgcn_global_load_lds(src, (lds_void *)lds_dst, 16, 0, 0);
}

// forward products of one 32-row block for both chain tiles: z[g][h] holds
// rows 16 h + 4 q + i (i = 0..3) of chain cl of tile g
template <int KC>
__device__ __forceinline__ void lr_fwd(const bf16x8 *L, int lane, const bf16x8 (&thi)[2][KC],
                                       const bf16x8 (&tlo)[2][KC], f32x4 (&z)[2][2]) {
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int h = 0; h < 2; ++h) z[g][h] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
    bf16x8 af[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) af[h] = L[(h * KC + kc) * 64 + lane];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        z[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[h], thi[g][kc], z[g][h], 0, 0, 0);
        z[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[h], tlo[g][kc], z[g][h], 0, 0, 0);
      }
  }
}

// Forward products of the next block (into zn) interleaved with the epilogue
// of the current one (from zc): residuals r (bf16, the backward B operand)
// and the per-chain log-density part.  The 4 KC MFMA pairs (theta hi, lo) and
// the 16 (row, chain) epilogue items are spread evenly over each other; an
// empty asm statement pins each item's results where it is written, so that
// the compiler keeps the vector-ALU work between the matrix-core instructions
// instead of sinking it to the end of the block (no instruction is emitted
// for it).  The two sides are independent, so a wavefront's matrix cores and
// vector ALU can work at the same time.
template <int KC>
__device__ __forceinline__ void lr_fwd_epi(const bf16x8 *L, int lane, const bf16x8 (&thi)[2][KC],
                                           const bf16x8 (&tlo)[2][KC], const f32x4 (&zc)[2][2], const float4 (&yl)[2],
                                           f32x4 (&zn)[2][2], bf16x8 (&rb)[2], float (&lq)[2]) {
  const float yv[2][4] = {{yl[0].x, yl[0].y, yl[0].z, yl[0].w}, {yl[1].x, yl[1].y, yl[1].z, yl[1].w}};
  bf16x8 af[KC][2];
#pragma unroll
  for (int kc = 0; kc < KC; ++kc)
#pragma unroll
    for (int h = 0; h < 2; ++h) af[kc][h] = L[(h * KC + kc) * 64 + lane];
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int h = 0; h < 2; ++h) zn[g][h] = f32x4{0.f, 0.f, 0.f, 0.f};
  float ab[2] = {0.f, 0.f}, prod[2] = {1.f, 1.f};
  float rr[2][8];
  constexpr int NG = 4 * KC;
#pragma unroll
  for (int k = 0; k < NG; ++k) {
    const int kc = k / 4, h = (k / 2) % 2, g = k % 2;
    zn[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[kc][h], thi[g][kc], zn[g][h], 0, 0, 0);
    zn[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[kc][h], tlo[g][kc], zn[g][h], 0, 0, 0);
    // epilogue items 16 k / NG .. 16 (k + 1) / NG - 1: row 16 eh + 4 q + ei of chain cl of tile eg
#pragma unroll
    for (int it = 16 * k / NG; it < 16 * (k + 1) / NG; ++it) {
      const int eg = it / 8, eh = (it / 4) % 2, ei = it % 4;
      const float zz = zc[eg][eh][ei];
      const float e = __builtin_amdgcn_exp2f(-fabsf(zz));
      const float ope = 1.0f + e;
      const float t = __builtin_amdgcn_rcpf(ope) - 0.5f;
      rr[eg][4 * eh + ei] = yv[eh][ei] - copysignf(t, zz);
      ab[eg] += fabsf(zz);
      prod[eg] *= ope;
      asm volatile("" : "+v"(rr[eg][4 * eh + ei]), "+v"(ab[eg]), "+v"(prod[eg]));
    }
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
#pragma unroll
    for (int j = 0; j < 8; ++j) rb[g][j] = (__bf16)rr[g][j];
    // prod lies in [1, 256]: the hardware log2 is accurate there
    lq[g] = fmaf(0.5f, ab[g], __builtin_amdgcn_logf(prod[g]));
  }
}

// backward products: the DT output tiles of 16 dims that hold dims < d (a
// tile wholly past d, e.g. the eighth for d = 100, is all padding)
template <int KC, int DT>
__device__ __forceinline__ void lr_bwd(const bf16x8 *L, int lane, const bf16x8 (&rb)[2], f32x4 (&gacc)[2][2 * KC]) {
#pragma unroll
  for (int dc = 0; dc < DT; ++dc) {
    const bf16x8 bfr = L[2 * KC * 64 + dc * 64 + lane];
#pragma unroll
    for (int g = 0; g < 2; ++g) gacc[g][dc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr, rb[g], gacc[g][dc], 0, 0, 0);
  }
}

template <int KC, int DT>
__global__ void __launch_bounds__(512, 2) k_lr_grad_bf16_pipe(LogregArgs a) {
  const bool go = lr_gate(a);
  constexpr int kThr = 512;
  constexpr int kFrag = 4 * KC * 64;      // 16-byte fragments per 32-row block
  constexpr int kPer = 2 * kFrag / kThr;   // fragments per thread per stage
  constexpr int kBuf = 2 * kFrag + 16;     // one buffer: two blocks' fragments + their 2 x 32 labels
  constexpr int kBlk = 2 * KC * 64;        // forward (or backward) fragments of one block
  __shared__ bf16x8 B0[kBuf], B1[kBuf], B2[kBuf];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int pg = wave & 3, rh = wave >> 2;
  const int q = lane >> 4, cl = lane & 15;
  const int64_t N = a.N, ld = a.ld, n = a.n;
  const int64_t mbase = (int64_t)blockIdx.x * 128 + pg * 32 + cl;  // chain of tile g: mbase + 16 g
  const float *X = static_cast<const float *>(a.x);
  const LrOffsets off = logreg_layout(1, n, a.d, N, ld, a.S);
  const bf16x8 *XF = reinterpret_cast<const bf16x8 *>(a.scratch + off.Xf);
  const bf16x8 *XB = reinterpret_cast<const bf16x8 *>(a.scratch + off.Xb);
  const bf16x8 *YF = reinterpret_cast<const bf16x8 *>(a.scratch + off.yf);  // labels, 4 floats per 16 bytes
  const int s = blockIdx.y;
  const int b0 = s * a.bps;
  const int b1 = (b0 + a.bps < a.NB) ? b0 + a.bps : a.NB;
  const int nit = (b1 - b0 + 1) / 2;
  // theta log2(e) of both chain tiles, split into bf16 hi + lo (B operand:
  // k slot 8q + j of chunk kc is coordinate 32 kc + 16 (j / 4) + 4 q + j % 4);
  // loaded before the first stage is issued
  // (every load is issued, from a clamped in-bounds address, and masked
  // afterwards, so that the sixteen loads are in flight together)
  float4 tv[2][KC][2];
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int64_t m = mbase + 16 * g;
    const int64_t mc = m < N ? m : N - 1;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int64_t d4 = 32 * kc + 16 * hh + 4 * q;
        tv[g][kc][hh] = *reinterpret_cast<const float4 *>(X + mc * ld + (d4 < ld ? d4 : 0));
      }
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const bool mv = mbase + 16 * g < N;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int hh = 0; hh < 2; ++hh)
        if (!(mv && 32 * kc + 16 * hh + 4 * q < ld)) tv[g][kc][hh] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  // Stage it holds blocks b0 + 2 it (half 0) and b0 + 2 it + 1 (half 1).
  // Fragment c of a buffer belongs to half c / kFrag; inside a block the
  // forward fragments precede the backward ones.  A wavefront's 64 fragments
  // of one instruction lie in one block, so the block test is uniform per
  // wavefront; lanes 0..15 of wavefront 0 also stage the labels.  A
  // fragment's source is a uniform base (advanced by two blocks per stage)
  // plus a loop-invariant per-thread offset.
  const bf16x8 *baseF = XF + (int64_t)b0 * kBlk, *baseB = XB + (int64_t)b0 * kBlk;
  int offk[kPer], halfk[kPer];
  bool fwdk[kPer], usek[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int c = tid + kThr * k;
    const int half = c / kFrag, f = c - half * kFrag;
    halfk[k] = half;
    fwdk[k] = f < kBlk;
    offk[k] = half * kBlk + (f < kBlk ? f : f - kBlk);
    // backward fragments of an all-padding output tile are never read
    usek[k] = f < kBlk || (f - kBlk) / 64 < DT;
  }
  auto stage = [&](int it, bf16x8 *buf) {
    if (it >= nit) return;
    const int64_t step = (int64_t)it * 2 * kBlk;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (usek[k] && b0 + 2 * it + halfk[k] < b1)
        lds_dma16((fwdk[k] ? baseF : baseB) + step + offk[k], buf + kThr * k + 64 * wave);
    }
    if (tid < 16) {
      const int64_t blk = b0 + 2 * it + (tid >> 3);
      if (blk < b1) lds_dma16(YF + blk * 8 + (tid & 7), buf + 2 * kFrag);
    }
  };
  // the gate, tested with theta's loads in flight and before any DMA into LDS
  if (!go) {
    __builtin_amdgcn_s_waitcnt(0);
    return;
  }
  stage(0, B0);
  stage(1, B1);
  bf16x8 thi[2][KC], tlo[2][KC];
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const float4 v = tv[g][kc][hh];
        const float f[4] = {v.x * 1.4426950408889634f, v.y * 1.4426950408889634f, v.z * 1.4426950408889634f,
                            v.w * 1.4426950408889634f};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const __bf16 hi = (__bf16)f[i];
          thi[g][kc][4 * hh + i] = hi;
          tlo[g][kc][4 * hh + i] = (__bf16)(f[i] - (float)hi);
        }
      }
  f32x4 gacc[2][2 * KC];
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int dc = 0; dc < 2 * KC; ++dc) gacc[g][dc] = f32x4{0.f, 0.f, 0.f, 0.f};
  double lacc[2] = {0.0, 0.0};
  // rows of the wavefront's last block past n: each contributed a factor 2 (log2 = 1)
  float padc = 0.f;
  {
    const int64_t blast = b0 + 2 * (nit - 1) + rh;
    const int64_t nv = n - 32 * blast;
    if (nit > 0 && blast < b1 && nv < 32)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) padc += (16 * h + 4 * q + i >= nv) ? 1.f : 0.f;
  }
  __syncthreads();  // stages 0 and 1 complete and visible
  f32x4 zc[2][2];
  lr_fwd<KC>(B0 + rh * kFrag, lane, thi, tlo, zc);
  // one iteration: stage it + 2 into Bn, forward of the next block from Bf,
  // epilogue and backward of the current block from Bc
  auto iter = [&](int it, const bf16x8 *Bc, const bf16x8 *Bf, bf16x8 *Bn) {
    // the current block's labels are read before the next stage's DMA is issued
    const float *Y = reinterpret_cast<const float *>(Bc + 2 * kFrag + 8 * rh);
    const float4 yl[2] = {*reinterpret_cast<const float4 *>(Y + 4 * q), *reinterpret_cast<const float4 *>(Y + 16 + 4 * q)};
    stage(it + 2, Bn);
    const bool use = b0 + 2 * it + rh < b1;
    f32x4 zn[2][2];
    bf16x8 rb[2];
    float lq[2];
    lr_fwd_epi<KC>(Bf + rh * kFrag, lane, thi, tlo, zc, yl, zn, rb, lq);
    // a block past the split's end (stale LDS, possibly not finite) contributes nothing (a
    // wavefront-uniform branch)
    if (use) {
      lr_bwd<KC, DT>(Bc + rh * kFrag, lane, rb, gacc);
      lacc[0] += (double)lq[0];
      lacc[1] += (double)lq[1];
    }
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int h = 0; h < 2; ++h) zc[g][h] = zn[g][h];
    // stage it + 2 complete and visible; every wavefront is done with Bc
    __syncthreads();
  };
  for (int it = 0; it < nit; it += 3) {
    iter(it, B0, B1, B2);
    if (it + 1 < nit) iter(it + 1, B1, B2, B0);
    if (it + 2 < nit) iter(it + 2, B2, B0, B1);
  }
  lacc[0] -= (double)padc;
  lacc[1] -= (double)padc;
  // half 1 hands its partial sums to half 0 through LDS (fixed order: half 0 + half 1);
  // a lane's four values of a tile are consecutive dims, moved as one 16-byte word
  // (tile g = 0 through B0, g = 1 through B1, the log-density sums through B2)
  f32x4 *const red[2] = {reinterpret_cast<f32x4 *>(B0), reinterpret_cast<f32x4 *>(B1)};
  double *lred = reinterpret_cast<double *>(B2);
  static_assert(kBuf >= 4 * 2 * KC * 64 && kBuf * 2 >= 4 * 2 * 64, "reduction buffers");
  if (rh == 1) {
#pragma unroll
    for (int g = 0; g < 2; ++g) {
#pragma unroll
      for (int dc = 0; dc < 2 * KC; ++dc) red[g][(pg * 2 * KC + dc) * 64 + lane] = gacc[g][dc];
      lred[(pg * 2 + g) * 64 + lane] = lacc[g];
    }
  }
  __syncthreads();
  if (rh == 0) {
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int64_t m = mbase + 16 * g;
      float *Gp = reinterpret_cast<float *>(a.scratch + off.Gp) + ((int64_t)s * N + m) * ld;
      if (m < N) {
#pragma unroll
        for (int dc = 0; dc < 2 * KC; ++dc) {
          const int64_t dd = 16 * dc + 4 * q;  // ld is a multiple of 8, so dd < ld covers dd .. dd + 3
          if (dd < ld) {
            const f32x4 v = gacc[g][dc] + red[g][(pg * 2 * KC + dc) * 64 + lane];
            *reinterpret_cast<f32x4 *>(Gp + dd) = v;
          }
        }
      }
      double la = lacc[g] + lred[(pg * 2 + g) * 64 + lane];
      la += __shfl_xor(la, 16);
      la += __shfl_xor(la, 32);
      // log2 units to natural log, with the sign of log p
      if (m < N && q == 0) reinterpret_cast<double *>(a.scratch + off.lp)[(int64_t)s * N + m] = -0.6931471805599453 * la;
    }
  }
}

// ---------------------------------------------------------------------------
// plain FP64 gradient on the FP64 matrix cores (v_mfma_f64_16x16x4_f64).
// grid (ceil(N/64), S), 256 threads = 4 wavefronts; wavefront w owns the 16
// chains 64 bx + 16 w .. + 15, and the workgroup walks the split's rows in
// tiles of 16, staged in LDS as FP64 rows (padded stride ld + 1 doubles).
// Lane layout of the instruction (A 16 x 4, B 4 x 16, D 16 x 16): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[l / 16 + 4 i]
// [l % 16], i = 0..3.
//   forward  z^T (rows x chains) += X[rows][k] theta[k][chains], 4 dims per
//            instruction: lane l holds z of chain l % 16 for rows l/16 + 4i;
//   epilogue r = y - sigmoid(z), y z - softplus(z) in FP64;
//   backward G (chains x dims) += r^T[chains][rows] X[rows][dims]: K-step i
//            takes rows i*4 .. i*4 + 3 as k = l / 16, exactly the rows the
//            lane already holds, so r feeds the A operand from registers.
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int KS>  // KS = ceil(d / 4) input-dim steps; d <= 128
__global__ void __launch_bounds__(256) k_lr_grad_f64_mfma(LogregArgs a) {
  const bool go = lr_gate(a);
  constexpr int DT = (4 * KS + 15) / 16;  // output tiles of 16 dims
  extern __shared__ double sm[];         // [2][16][ldl] rows, then [2][16] labels
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lo = lane & 15, hi = lane >> 4;
  const int64_t N = a.N, ld = a.ld, d = a.d, n = a.n;
  const int ldl = (int)ld + 1;
  double *Xs = sm, *Ys = sm + 2 * 16 * ldl;
  const double *x = static_cast<const double *>(a.x);
  const double *X = static_cast<const double *>(a.X);
  const int64_t m = (int64_t)blockIdx.x * 64 + 16 * wave + lo;  // chain of the B operand / backward A operand
  // theta as the forward B operand: step s supplies theta[m][4 s + hi]
  double th[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int64_t e = 4 * k + hi;
    th[k] = (m < N && e < d) ? x[m * ld + e] : 0.0;
  }
  if (!go) {
    __builtin_amdgcn_s_waitcnt(0);
    return;
  }
  f64x4 gacc[DT];
#pragma unroll
  for (int t = 0; t < DT; ++t) gacc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  double lacc = 0.0;
  const int s = blockIdx.y;
  const int64_t r0 = (int64_t)s * a.bps * 32;
  int64_t r1 = r0 + (int64_t)a.bps * 32;
  if (r1 > n) r1 = n;
  const int64_t ntile = (r1 - r0 + 15) / 16;
  // staging of row tile tt into buffer b: 16 rows x ld doubles (zero past d and n), and the labels.
  // Thread tid copies row tid / 16, columns tid % 16 + 16 j; the loads use clamped in-range indices
  // and the bounds enter as 0 / 1 factors (X is finite), so none of them waits in a branch of its own.
  auto stage = [&](int64_t tt, int b) {
    const int64_t rb = r0 + 16 * tt;
    const int rr = tid >> 4;
    const int64_t row = rb + rr;
    const double rf = row < r1 ? 1.0 : 0.0;
    const double *src = X + (row < r1 ? row : r1 - 1) * d;
    double *dst = Xs + (b * 16 + rr) * ldl;
    for (int e = tid & 15; e < (int)ld; e += 16) dst[e] = src[e < d ? e : d - 1] * (e < d ? rf : 0.0);
    if (tid < 16) Ys[b * 16 + tid] = (rb + tid < r1) ? a.y[rb + tid] : 0.0;
  };
  if (ntile > 0) stage(0, 0);
  __syncthreads();
  // softplus(z) = max(z, 0) + log(1 + e^{-|z|}): the factors 1 + e^{-|z|} in (1, 2] of the lane's rows
  // are multiplied and their logarithm taken once per 8 tiles (32 factors, below 2^32); rounding each
  // factor to FP64 costs at most 2^-53 absolute in its logarithm
  double pf = 1.0;
  for (int64_t tt = 0; tt < ntile; ++tt) {
    const int b = (int)(tt & 1);
    if (tt + 1 < ntile) stage(tt + 1, b ^ 1);
    const double *T = Xs + b * 16 * ldl;
    // forward: A = X[row lo][4 k + hi], even and odd K-steps in two accumulators (two dependency chains)
    f64x4 z0 = f64x4{0.0, 0.0, 0.0, 0.0}, z1 = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KS; k += 2) {
      z0 = __builtin_amdgcn_mfma_f64_16x16x4f64(T[lo * ldl + 4 * k + hi], th[k], z0, 0, 0, 0);
      if (k + 1 < KS)
        z1 = __builtin_amdgcn_mfma_f64_16x16x4f64(T[lo * ldl + 4 * (k + 1) + hi], th[k + 1], z1, 0, 0, 0);
    }
    const f64x4 z = z0 + z1;
    // epilogue on the lane's rows hi + 4 i of chain m
    const int64_t rb = r0 + 16 * tt;
    double rv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = hi + 4 * i;
      const double zz = z[i];
      const double yv = Ys[b * 16 + rr];
      const double ez = exp(-fabs(zz));
      const double q = 1.0 + ez;
      const double sg = (zz >= 0.0 ? 1.0 : ez) / q;
      const bool ok = rb + rr < r1;
      rv[i] = ok ? yv - sg : 0.0;
      lacc += ok ? yv * zz - fmax(zz, 0.0) : 0.0;
      pf *= ok ? q : 1.0;
    }
    if ((tt & 7) == 7) {
      lacc -= log(pf);
      pf = 1.0;
    }
    // backward: K-step i takes the rows hi + 4 i (A = r from registers, B = X[row][16 t + lo])
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double *Tr = T + (hi + 4 * i) * ldl;
#pragma unroll
      for (int t = 0; t < DT; ++t) {
        const int e = 16 * t + lo;
        gacc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(rv[i], e < ld ? Tr[e] : 0.0, gacc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const LrOffsets off = logreg_layout(0, n, d, N, ld, a.S);
  double *Gp = reinterpret_cast<double *>(a.scratch + off.Gp);
  // lane l holds G[chain 16 w + hi + 4 i][dim 16 t + lo]
#pragma unroll
  for (int t = 0; t < DT; ++t) {
    const int64_t e = 16 * t + lo;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t mc = (int64_t)blockIdx.x * 64 + 16 * wave + hi + 4 * i;
      if (mc < N && e < ld) Gp[((int64_t)s * N + mc) * ld + e] = gacc[t][i];
    }
  }
  lacc -= log(pf);
  // log p partial of chain m: the lanes with equal lo hold its rows (xor over hi)
  lacc += __shfl_xor(lacc, 16);
  lacc += __shfl_xor(lacc, 32);
  if (m < N && hi == 0) reinterpret_cast<double *>(a.scratch + off.lp)[(int64_t)s * N + m] = lacc;
}

// ---------------------------------------------------------------------------
// per-chain update kernels: one team of T <= 16 lanes per chain (64, 128 or
// 256 threads), lane r holding the Q octs r + q T (q < Q) of the chain
// ---------------------------------------------------------------------------
template <class Real, int Q>
__device__ __forceinline__ void lr_grad_sum(const LogregArgs &a, const LrOffsets &off, int64_t m, int r, int T,
                                            bool act, const Real (&x)[Q][8], Real (&g)[Q][8], double &lps) {
  const Real *Gp = reinterpret_cast<const Real *>(a.scratch + off.Gp);
  const double *lp = reinterpret_cast<const double *>(a.scratch + off.lp);
  Real acc[Q][8] = {};
  lps = 0.0;
  // splits in order, four at a time: the four loads are issued before the
  // first of them is used, so the split sum costs ~S/4 memory latencies
  const int S = act ? a.S : 0;
  bool mine[Q];
  int64_t e0[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    e0[q] = 8 * (int64_t)(r + q * T);
    mine[q] = e0[q] < a.d;
  }
  int s = 0;
  for (; s + 4 <= S; s += 4) {
    Real v[4][Q][8];
    double l[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
        if (mine[q]) ld8<Real>(Gp + ((int64_t)(s + k) * a.N + m) * a.ld + e0[q], v[k][q]);
      l[k] = lp[(int64_t)(s + k) * a.N + m];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
        if (mine[q])
#pragma unroll
          for (int i = 0; i < 8; ++i) acc[q][i] += v[k][q][i];
      lps += l[k];
    }
  }
  for (; s < S; ++s) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (mine[q]) {
        Real v[8];
        ld8<Real>(Gp + ((int64_t)s * a.N + m) * a.ld + e0[q], v);
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[q][i] += v[i];
      }
    lps += lp[(int64_t)s * a.N + m];
  }
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int i = 0; i < 8; ++i)
      g[q][i] = (e0[q] + i < a.d) ? acc[q][i] - (a.prior ? x[q][i] : Real(0)) : Real(0);
}

// The lane's share of the log-density terms that depend on theta alone: the
// N(0, I) prior -|theta|^2 / 2 and, for the bf16 gradient (whose split sums
// leave it out), sum_n (y_n - 1/2) z_n = theta . (X^T (y - 1/2)) in FP64.
template <class Real, int Q>
__device__ __forceinline__ double lr_theta_terms(const LogregArgs &a, const LrOffsets &off, int r, int T,
                                                 const Real (&x)[Q][8]) {
  double v = 0.0;
  if (a.prior) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) v -= 0.5 * (double)x[q][i] * (double)x[q][i];
  }
  if (a.wy_term) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t e0 = 8 * (int64_t)(r + q * T);
      if (e0 < a.d) {
        const double *wy = reinterpret_cast<const double *>(a.scratch + off.wy) + e0;
#pragma unroll
        for (int i = 0; i < 8; ++i) v += (double)x[q][i] * wy[i];
      }
    }
  }
  return v;
}

template <class Real, int Q>
__global__ void __launch_bounds__(256) k_lr_update(LogregArgs a) {
  const bool go = lr_gate(a);
#define LR_GATE_TEST()               \
  do {                               \
    if (!go) {                       \
      __builtin_amdgcn_s_waitcnt(0); \
      return;                        \
    }                                \
  } while (0)
  extern __shared__ double smem[];
  double *red = smem;
  const int T = a.T;
  const int team = threadIdx.x / T, r = threadIdx.x - team * T;
  int slot = 0;
  const int64_t N = a.N, d = a.d, ld = a.ld;
  const int64_t m = (int64_t)blockIdx.x * a.tpw + team;
  const bool act = m < N;
  const double dm1 = (double)(d - 1);
  const LrOffsets off = logreg_layout(sizeof(Real) == 8 ? 0 : 1, a.n, d, N, ld, a.S);
  double *sc = reinterpret_cast<double *>(a.scratch + off.sc);
  double *sc_l0 = sc, *sc_lprev = sc + N, *sc_D = sc + 2 * N, *sc_dk = sc + 3 * N;
  Real *X = static_cast<Real *>(a.x);
  Real *U = static_cast<Real *>(a.u);
  Real *Gc = static_cast<Real *>(a.g);
  Real *X0 = reinterpret_cast<Real *>(a.scratch + off.x0);
  Real *G0 = reinterpret_cast<Real *>(a.scratch + off.g0);
  const DevHyper *H = a.hyp;
  const double eps = H->eps;
  const uint64_t t = (uint64_t)H->t;
  const double h = 0.5 * eps;
  Real x[Q][8], u[Q][8], g[Q][8], z[Q][8];
  load_row<Real, Q>(X + m * ld, r, T, d, act, x);
  const int mode = a.mode;

  if (mode == LR_EVAL) {
    // log p and gradient at the caller's positions (a.x): split sums plus the prior
    double lps;
    lr_grad_sum<Real, Q>(a, off, m, r, T, act, x, g, lps);
    LR_GATE_TEST();
    double v[1] = {lr_theta_terms<Real, Q>(a, off, r, T, x)};
    team_sum<1>(v, T, red, slot);
    if (act) {
      if (a.g_out) store_row<Real, Q>(static_cast<Real *>(a.g_out) + m * ld, r, T, d, g);
      if (r == 0) a.logp_out[m] = lps + v[0];
    }
    return;
  }

  if (mode == LR_INIT || mode == LR_POST) {
    double S[4][Q][8] = {};
    // every global load of this stage is issued before the first dependent use
    double K[Q][8];
    if (mode == LR_POST) {
      load_shift<Q>(a.shiftK, r, T, d, K);
      load_row<Real, Q>(U + m * ld, r, T, d, act, u);
    }
    double lps;
    lr_grad_sum<Real, Q>(a, off, m, r, T, act, x, g, lps);
    LR_GATE_TEST();
    if (mode == LR_INIT) {
      lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, 0, TAG_INIT_DIR, 0, z);
      double v[3] = {lr_theta_terms<Real, Q>(a, off, r, T, x), 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          v[1] += (double)g[q][i] * (double)g[q][i];
          v[2] += (double)z[q][i] * (double)z[q][i];
        }
      team_sum<3>(v, T, red, slot);
      const double l1 = lps + v[0];
      if (a.u0) {
        load_row<Real, Q>(static_cast<const Real *>(a.u0) + m * ld, r, T, d, act, u);
      } else {
        const double gn = sqrt(v[1]);
        const bool useg = gn > 0.0 && isfinite(gn);
        const Real scl = (Real)(1.0 / (useg ? gn : sqrt(v[2])));
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int i = 0; i < 8; ++i) u[q][i] = (useg ? g[q][i] : z[q][i]) * scl;
      }
      if (act) {
        store_row<Real, Q>(X + m * ld, r, T, d, x);
        store_row<Real, Q>(U + m * ld, r, T, d, u);
        store_row<Real, Q>(Gc + m * ld, r, T, d, g);
        if (r == 0) {
          a.logp[m] = l1;
          a.delta[m] = 0.0;
          a.acc[m] = 0.0;
        }
        const double K0[Q][8] = {};
        accumulate_stats<Real, Q>(S, K0, x, g);
      }
    } else {
      const double Lm = H->L;
      const Real c1 = (Real)exp(-h / Lm), c2 = (Real)(sqrt(-expm1(-2.0 * h / Lm)) / sqrt((double)d));
      double v[3] = {lr_theta_terms<Real, Q>(a, off, r, T, x), 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          v[1] += (double)g[q][i] * (double)g[q][i];
          v[2] += (double)g[q][i] * (double)u[q][i];
        }
      team_sum<3>(v, T, red, slot);
      const double l1 = lps + v[0];
      const BMap b2 = b_map_dyn<Real>(a.dyn, v[1], v[2], h, dm1);
      lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, t, TAG_O_SECOND, 0, z);
      double w1[1] = {0.0};
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const Real w = c1 * ((Real)b2.A * u[q][i] + (Real)b2.Bg * g[q][i]) + c2 * z[q][i];
          u[q][i] = w;
          w1[0] += (double)w * (double)w;
        }
      team_sum<1>(w1, T, red, slot);
      const Real inw = (Real)refresh_scale(a.dyn, w1[0]);
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) u[q][i] *= inw;
      if (act) {
        store_row<Real, Q>(U + m * ld, r, T, d, u);
        store_row<Real, Q>(Gc + m * ld, r, T, d, g);
        if (r == 0) {
          a.logp[m] = l1;
          a.delta[m] = (sc_l0[m] - l1) + sc_dk[m] + b2.dK;
        }
        accumulate_stats<Real, Q>(S, K, x, g);
      }
    }
    write_partials<Real, Q>(a.partials, d, ld, S, red + 2 * kRedSlots, T, r);
    return;
  }

  if (mode == LR_PRE) {
    const double Lm = H->L;
    const Real c1 = (Real)exp(-h / Lm), c2 = (Real)(sqrt(-expm1(-2.0 * h / Lm)) / sqrt((double)d));
    load_row<Real, Q>(U + m * ld, r, T, d, act, u);
    load_row<Real, Q>(Gc + m * ld, r, T, d, act, g);
    lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, t, TAG_O_FIRST, 0, z);
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const Real w = c1 * u[q][i] + c2 * z[q][i];
        u[q][i] = w;
        v[0] += (double)w * (double)w;
        v[1] += (double)g[q][i] * (double)w;
        v[2] += (double)g[q][i] * (double)g[q][i];
      }
    team_sum<3>(v, T, red, slot);
    const double inw = refresh_scale(a.dyn, v[0]);
    const BMap b1 = b_map_dyn<Real>(a.dyn, v[2], v[1] * inw, h, dm1);
    const Real A1 = (Real)(b1.A * inw), B1 = (Real)b1.Bg, epsR = (Real)eps;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        u[q][i] = A1 * u[q][i] + B1 * g[q][i];
        x[q][i] += epsR * u[q][i];
      }
    LR_GATE_TEST();
    if (act) {
      store_row<Real, Q>(X + m * ld, r, T, d, x);
      store_row<Real, Q>(U + m * ld, r, T, d, u);
      if (r == 0) {
        sc_l0[m] = a.logp[m];
        sc_dk[m] = b1.dK;
      }
    }
    return;
  }

  // adjusted phase: preconditioned MAMS trajectory, one stage per launch
  const double Lp = a.Lp_factor * (double)a.n_traj * eps;
  const Real c1 = (Real)exp(-h / Lp), c2 = (Real)(sqrt(-expm1(-2.0 * h / Lp)) / sqrt((double)d));
  Real sg[Q][8];
  load_row<Real, Q>(static_cast<const Real *>(a.sigma), r, T, d, true, sg);
  double D = 0.0, lprev = 0.0;

  // first half of a step: O_{eps/2}(j), B_{b0 eps}, A_{a0 eps}
  auto step_start = [&](int j) {
    lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, t, TAG_O_FIRST, (uint32_t)j, z);
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const Real w = c1 * u[q][i] + c2 * z[q][i];
        const Real gt = sg[q][i] * g[q][i];
        u[q][i] = w;
        v[0] += (double)w * (double)w;
        v[1] += (double)gt * (double)w;
        v[2] += (double)gt * (double)gt;
      }
    team_sum<3>(v, T, red, slot);
    const double inw = refresh_scale(a.dyn, v[0]);
    const BMap b = b_map_dyn<Real>(a.dyn, v[2], v[1] * inw, a.cb0 * eps, dm1);
    D += b.dK;
    const Real Ab = (Real)(b.A * inw), Bb = (Real)b.Bg, ha = (Real)(a.ca0 * eps);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        u[q][i] = Ab * u[q][i] + Bb * sg[q][i] * g[q][i];
        x[q][i] += ha * sg[q][i] * u[q][i];
      }
  };

  if (mode == LR_MBEGIN) {
    load_row<Real, Q>(Gc + m * ld, r, T, d, act, g);
    LR_GATE_TEST();
    if (act) {
      store_row<Real, Q>(X0 + m * ld, r, T, d, x);
      store_row<Real, Q>(G0 + m * ld, r, T, d, g);
    }
    const double l0 = act ? a.logp[m] : 0.0;
    lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, t, TAG_FULL_REFRESH, 0, z);
    double v1[1] = {0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) v1[0] += (double)z[q][i] * (double)z[q][i];
    team_sum<1>(v1, T, red, slot);
    const Real iz = (Real)full_refresh_scale(a.dyn, v1[0], d);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) u[q][i] = z[q][i] * iz;
    step_start(0);
    if (act) {
      store_row<Real, Q>(X + m * ld, r, T, d, x);
      store_row<Real, Q>(U + m * ld, r, T, d, u);
      if (r == 0) {
        sc_l0[m] = l0;
        sc_lprev[m] = l0;
        sc_D[m] = D;
      }
    }
    return;
  }

  // LR_MSTEP: consume gradient k of step j
  load_row<Real, Q>(U + m * ld, r, T, d, act, u);
  double lps;
  lr_grad_sum<Real, Q>(a, off, m, r, T, act, x, g, lps);
  LR_GATE_TEST();
  double v[3] = {lr_theta_terms<Real, Q>(a, off, r, T, x), 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const Real gt = sg[q][i] * g[q][i];
      v[1] += (double)gt * (double)gt;
      v[2] += (double)gt * (double)u[q][i];
    }
  team_sum<3>(v, T, red, slot);
  const double lnew = lps + v[0];
  D = (act ? sc_D[m] + (sc_lprev[m] - lnew) : 0.0);
  lprev = lnew;
  const int k = a.k, j = a.j;
  {
    const BMap b = b_map_dyn<Real>(a.dyn, v[1], v[2], a.cbk * eps, dm1);
    D += b.dK;
    const Real Ab = (Real)b.A, Bb = (Real)b.Bg;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) u[q][i] = Ab * u[q][i] + Bb * sg[q][i] * g[q][i];
  }
  if (k + 1 < a.cK - 1) {
    const Real ha = (Real)(a.cak * eps);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) x[q][i] += ha * sg[q][i] * u[q][i];
  } else {
    lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, t, TAG_O_SECOND, (uint32_t)j, z);
    double w1[1] = {0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const Real w = c1 * u[q][i] + c2 * z[q][i];
        u[q][i] = w;
        w1[0] += (double)w * (double)w;
      }
    team_sum<1>(w1, T, red, slot);
    const Real inw = (Real)refresh_scale(a.dyn, w1[0]);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) u[q][i] *= inw;
    if (j + 1 < a.n_traj) {
      step_start(j + 1);
    } else {
      // Metropolis test on the whole trajectory's energy error
      const double wacc = exp(-D);
      const bool nanD = (D != D);
      const double am = nanD ? 0.0 : (wacc < 1.0 ? wacc : 1.0);
      const double U01 = mh_uniform(a.seed, (uint64_t)m, t);
      const bool accept = !nanD && (U01 < wacc);
      if (act) {
        if (accept) {
          store_row<Real, Q>(X + m * ld, r, T, d, x);
          store_row<Real, Q>(Gc + m * ld, r, T, d, g);
          if (r == 0) a.logp[m] = lnew;
        } else {
          Real x0[Q][8], g0[Q][8];
          load_row<Real, Q>(X0 + m * ld, r, T, d, true, x0);
          load_row<Real, Q>(G0 + m * ld, r, T, d, true, g0);
          store_row<Real, Q>(X + m * ld, r, T, d, x0);
          store_row<Real, Q>(Gc + m * ld, r, T, d, g0);
          if (r == 0) a.logp[m] = sc_l0[m];
        }
        if (r == 0) {
          a.acc[m] = am;
          a.delta[m] = D;
        }
      }
      return;
    }
  }
  if (act) {
    store_row<Real, Q>(X + m * ld, r, T, d, x);
    store_row<Real, Q>(U + m * ld, r, T, d, u);
    store_row<Real, Q>(Gc + m * ld, r, T, d, g);
    if (r == 0) {
      sc_D[m] = D;
      sc_lprev[m] = lprev;
    }
  }
}
#undef LR_GATE_TEST

// ---------------------------------------------------------------------------
hipError_t launch_logreg_pack(const LogregArgs &a, hipStream_t s) {
  const int KC = a.KC, NB = a.NB;
  const LrOffsets off = logreg_layout(1, a.n, a.d, a.N, a.ld, a.S);
  const int64_t total = (int64_t)NB * 2 * KC * 64 * 2 + (int64_t)NB * 32 + a.ld;
  hipLaunchKernelGGL(k_lr_pack, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     static_cast<const unsigned short *>(a.X), a.y, a.n, a.d, a.ld, KC, NB,
                     reinterpret_cast<unsigned short *>(a.scratch + off.Xf),
                     reinterpret_cast<unsigned short *>(a.scratch + off.Xb), reinterpret_cast<float *>(a.scratch + off.yf),
                     reinterpret_cast<double *>(a.scratch + off.wy));
  return hipGetLastError();
}

hipError_t launch_logreg_grad(int prec, const LogregArgs &a, hipStream_t s) {
  if (prec == 0) {
    const int KS = (int)((a.d + 3) / 4);
    if (KS < 1 || KS > 32) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.N + 63) / 64), (unsigned)a.S);
    const size_t shm = ((size_t)2 * 16 * (a.ld + 1) + 32) * sizeof(double);
    typedef void (*Fn)(LogregArgs);
    static const Fn fns[32] = {
        k_lr_grad_f64_mfma<1>,  k_lr_grad_f64_mfma<2>,  k_lr_grad_f64_mfma<3>,  k_lr_grad_f64_mfma<4>,
        k_lr_grad_f64_mfma<5>,  k_lr_grad_f64_mfma<6>,  k_lr_grad_f64_mfma<7>,  k_lr_grad_f64_mfma<8>,
        k_lr_grad_f64_mfma<9>,  k_lr_grad_f64_mfma<10>, k_lr_grad_f64_mfma<11>, k_lr_grad_f64_mfma<12>,
        k_lr_grad_f64_mfma<13>, k_lr_grad_f64_mfma<14>, k_lr_grad_f64_mfma<15>, k_lr_grad_f64_mfma<16>,
        k_lr_grad_f64_mfma<17>, k_lr_grad_f64_mfma<18>, k_lr_grad_f64_mfma<19>, k_lr_grad_f64_mfma<20>,
        k_lr_grad_f64_mfma<21>, k_lr_grad_f64_mfma<22>, k_lr_grad_f64_mfma<23>, k_lr_grad_f64_mfma<24>,
        k_lr_grad_f64_mfma<25>, k_lr_grad_f64_mfma<26>, k_lr_grad_f64_mfma<27>, k_lr_grad_f64_mfma<28>,
        k_lr_grad_f64_mfma<29>, k_lr_grad_f64_mfma<30>, k_lr_grad_f64_mfma<31>, k_lr_grad_f64_mfma<32>};
    hipLaunchKernelGGL(fns[KS - 1], grid, dim3(256), shm, s, a);
    return hipGetLastError();
  }
  if (a.KC < 1 || a.KC > 4) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((a.N + 127) / 128), (unsigned)a.S);
  // output tiles of 16 dims holding dims < d: 2 KC - 1 or 2 KC
  const bool odd = (a.d + 15) / 16 < 2 * a.KC;
  void (*const fns[4][2])(LogregArgs) = {{k_lr_grad_bf16_pipe<1, 2>, k_lr_grad_bf16_pipe<1, 1>},
                                         {k_lr_grad_bf16_pipe<2, 4>, k_lr_grad_bf16_pipe<2, 3>},
                                         {k_lr_grad_bf16_pipe<3, 6>, k_lr_grad_bf16_pipe<3, 5>},
                                         {k_lr_grad_bf16_pipe<4, 8>, k_lr_grad_bf16_pipe<4, 7>}};
  void (*fn)(LogregArgs) = fns[a.KC - 1][odd ? 1 : 0];
  LogregArgs arg = a;
  void *args[] = {&arg};
  return hipLaunchKernel(reinterpret_cast<const void *>(fn), grid, dim3(512), args, 0, s);
}

hipError_t launch_logreg_update(int prec, int Q, const LogregArgs &a, int grid, int block, size_t shmem,
                                hipStream_t s) {
  typedef void (*Fn)(LogregArgs);
  static const Fn fd[4] = {k_lr_update<double, 1>, k_lr_update<double, 2>, k_lr_update<double, 3>,
                           k_lr_update<double, 4>};
  static const Fn ff[4] = {k_lr_update<float, 1>, k_lr_update<float, 2>, k_lr_update<float, 3>,
                           k_lr_update<float, 4>};
  if (Q < 1 || Q > 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL((prec == 0 ? fd : ff)[Q - 1], dim3(grid), dim3(block), shmem, s, a);
  return hipGetLastError();
}

}  // namespace laps
