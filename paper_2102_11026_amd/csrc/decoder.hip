// Decoder kernels: collective complex-step right contractions (Sec. 4.3) as
// MFMA GEMMs over stacked jet channels with the activation's derivative chain
// fused into the epilogue, and complex-step backpropagation (Sec. 4.4).
//
// Multicomplex arithmetic in the h -> 0 limit.  A forward perturbation
// q + h e_j i1 + h dq i2 + h dq i3 (and q + h e_j i1 + h qdot i4) is carried
// as real channels, each multicomplex component divided by h^order (a jet).
// Because the weights are real, a fully connected layer acts on every
// channel separately (the block structure of the Cauchy-Riemann form,
// Sec. 6.7), so all channels of all perturbations are the columns of one
// GEMM.  An activation sigma of x = x0 + x1 i1 + x2 i2 + x2 i3 + x4 i4 + ...
// expands by the multinomial Taylor series (eq. mc_taylor); keeping every
// component the contractions need gives, with sigma^(k) at x0,
//   y1   = s1 x1                 y2  = s1 x2          y4 = s1 x4
//   y12  = s1 x12 + s2 x1 x2     y14 = s1 x14 + s2 x1 x4
//   y23  = s1 x23 + s2 x2 x2
//   y123 = s1 x123 + s2 (x1 x23 + 2 x2 x12) + s3 x1 x2 x2
// The dropped components are O(h^2) relative to those kept, below rounding
// for h = 1e-20 (FP64) and h = 1e-10 (FP32 jets), so the channels equal the
// complex-step quotients of eq. cfd / eq. mcfd_hessian up to rounding.
//
// Complex-step backpropagation (Sec. 4.4): the forward pass from q + h e_j i
// stores, per hidden neuron, the pre-activation x0 + h x1_j i (the value and
// e_j-tangent channels above).  BP of g = s . m(q) in complex arithmetic
// multiplies the adjoint by sigma'(x0 + h x1 i) = s1 + h s2 x1 i, so with the
// adjoint zb0 + h zb1_j i:  xb0 = s1 zb0,  xb1_j = s1 zb1_j + s2 x1_j zb0.
// At the input Re = m_q^T s and Im/h = column j of s . H.
//
// GEMM tiling for gfx950.  The hidden layers are small (<= 1024 x 1024, 16..128
// channel columns), so a launch is latency-bound: each 16-row output tile is
// owned by one block of NW wavefronts that split the K dimension, each wave
// issuing its loads for up to four K-steps before its MFMAs, and the NW
// partial tiles are added in LDS in wave order (deterministic).  The output
// layer (N x K with N up to 1.5e5) is bandwidth-bound: every wave owns 16
// rows, issues all of its weight loads first and reads the folded
// activations from LDS.
#include "nmr_internal.h"

#include <type_traits>

namespace nmr {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline void act_jet(int act, T x, T& y, T& d1, T& d2, T& d3) {
  if (act == ACT_TANH) {
    T t = tanh(x);
    y = t;
    d1 = T(1) - t * t;
    d2 = T(-2) * t * d1;
    d3 = T(-2) * d1 * (T(1) - T(3) * t * t);
  } else if (act == ACT_ELU) {
    if (x > T(0)) {
      y = x; d1 = T(1); d2 = T(0); d3 = T(0);
    } else {
      T e = exp(x);
      y = expm1(x); d1 = e; d2 = e; d3 = e;
    }
  } else if (act == ACT_SIN) {
    T s = sin(x), c = cos(x);
    y = s; d1 = c; d2 = -s; d3 = -c;
  } else {
    y = x; d1 = T(1); d2 = T(0); d3 = T(0);
  }
}

template <typename T>
__device__ inline void act_d12(int act, T x, T& d1, T& d2) {
  T y, d3;
  act_jet(act, x, y, d1, d2, d3);
}

template <typename V>
__device__ inline V zero_of() {
  V v;
  __builtin_memset(&v, 0, sizeof(V));
  return v;
}

template <typename T> struct vec4;
template <> struct vec4<float> { typedef float4 type; };
template <> struct vec4<double> { typedef double4 type; };

// One layer of the decoder as a launch sees it, passed by value: everything
// a kernel reads from it arrives with the first kernel-argument load, with
// no index by a runtime layer number into the decoder's tables.
struct LayerArgs {
  const void* W;   // W_l, [m_outp][m_inp] (padded, K contiguous)
  const void* b;   // b_l, [m_out]
  const void* WT;  // W_l^T, [m_inp][m_outp] (hidden layers only)
  int l, L, act;
  int m_in, m_inp, m_out, m_outp;  // true and padded input / output widths
  int bf16;                        // BF16 decoder: activations and adjoints stored as BF16
};

static LayerArgs layer_args(const DecoderDev& d, int l) {
  LayerArgs a;
  a.W = d.W[l];
  a.b = d.b[l];
  a.WT = (l < d.L - 1) ? d.WT[l] : nullptr;
  a.l = l;
  a.L = d.L;
  a.act = d.act;
  a.m_in = d.w[l];
  a.m_inp = d.wp[l];
  a.m_out = d.w[l + 1];
  a.m_outp = d.wp[l + 1];
  a.bf16 = d.prec == PREC_BF16 ? 1 : 0;
  return a;
}

template <typename TW> struct kstep { static constexpr int v = 16; };
template <> struct kstep<__bf16> { static constexpr int v = 32; };
template <> struct kstep<double> { static constexpr int v = 4; };

// waves per split-K block: keep the partial tiles within 32 KB of LDS
template <typename T, int NCB>
struct splitk_waves { static constexpr int v = (NCB * (int)sizeof(T) <= 16) ? 8 : 4; };

// ---------------------------------------------------------------------------
// One wave: partial 16 x (NCB*16) tile over k in [kb, ke).  A is [16][lda]
// (K contiguous), B is read as 4 consecutive K entries of column c through
// bload(c, k).  acc[cb][i] = D[4*(lane/16) + i][cb*16 + lane%16].
// ---------------------------------------------------------------------------
template <int NCB, typename BL>
__device__ inline void mfma_range(const float* __restrict__ A, int lda, int kb, int ke, BL bload,
                                  f32x4 (&acc)[NCB]) {
  constexpr int PF = NCB <= 4 ? 4 : 2;  // K-steps whose loads are issued together
  const int lane = threadIdx.x & 63;
  const int rA = lane & 15, g = lane >> 4;
  const float* ap = A + (size_t)rA * lda + 4 * g;
  for (int k0 = kb; k0 < ke; k0 += 16 * PF) {
    float4 a[PF];
    float4 b[PF][NCB];
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int k = k0 + 16 * t;
      if (k < ke) {
        a[t] = ldg<float4>(ap + k);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[t][cb] = bload(cb * 16 + rA, k + 4 * g);
      } else {
        a[t] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[t][cb] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int t = 0; t < PF; ++t)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t].x, b[t][cb].x, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t].y, b[t][cb].y, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t].z, b[t][cb].z, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t].w, b[t][cb].w, acc[cb], 0, 0, 0);
      }
  }
}

__device__ inline bf16x8 to_bf16x8(float4 lo, float4 hi) {
  bf16x8 b;
  b[0] = (__bf16)lo.x; b[1] = (__bf16)lo.y; b[2] = (__bf16)lo.z; b[3] = (__bf16)lo.w;
  b[4] = (__bf16)hi.x; b[5] = (__bf16)hi.y; b[6] = (__bf16)hi.z; b[7] = (__bf16)hi.w;
  return b;
}

// K entries k .. k + 7 of B column c as a BF16 fragment: loaded as they are
// from a BF16 operand (a BF16 decoder's hidden activations and adjoints are
// stored rounded), or rounded here from two FP32 loads (the decoder input).
// Either way each value is rounded once, from the same FP32 value.
template <typename BL>
__device__ inline bf16x8 bfrag(BL& bload, int c, int k) {
  if constexpr (std::is_same<decltype(bload(c, k)), bf16x8>::value) return bload(c, k);
  else return to_bf16x8(bload(c, k), bload(c, k + 4));
}

template <int NCB, typename BL>
__device__ inline void mfma_range(const __bf16* __restrict__ A, int lda, int kb, int ke, BL bload,
                                  f32x4 (&acc)[NCB]) {
  constexpr int PF = NCB <= 4 ? 4 : 2;
  const int lane = threadIdx.x & 63;
  const int rA = lane & 15, g = lane >> 4;
  const __bf16* ap = A + (size_t)rA * lda + 8 * g;
  for (int k0 = kb; k0 < ke; k0 += 32 * PF) {
    bf16x8 a[PF];
    bf16x8 b[PF][NCB];
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int k = k0 + 32 * t;
      if (k < ke) {
        a[t] = ldg<bf16x8>(ap + k);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[t][cb] = bfrag(bload, cb * 16 + rA, k + 8 * g);
      } else {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        a[t] = to_bf16x8(z, z);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[t][cb] = to_bf16x8(z, z);
      }
    }
#pragma unroll
    for (int t = 0; t < PF; ++t)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], b[t][cb], acc[cb], 0, 0, 0);
  }
}

// Split-K tile over IB instance slots: the NW waves of a block are IB slots x
// KSPL = NW / IB K-slices.  Wave w computes the partial 16 x (NCB*16) tile of
// slot w / KSPL over its slice of K (A is [16][lda], K contiguous; B through
// bload(c, k)), and the slices of each slot are added in slice order into
// S[slot][c][r] (c = column < NCB*16, r = row < 16).  A slot that is not in
// use (use == false) contributes zeros; every wave reaches every barrier.
template <typename T, typename TW, int NCB, int NW, int IB, typename BL>
__device__ inline void gemm_splitk(const TW* __restrict__ A, int lda, int K, bool use, BL bload,
                                   T (*S)[NCB * 16][17], T (*red)[NCB * 16][16]) {
  constexpr int KSPL = NW / IB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ks = wave % KSPL;
  constexpr int KS = kstep<TW>::v;
  const int nks = K / KS;
  const int per = (nks + KSPL - 1) / KSPL;
  const int kb = min(K, ks * per * KS), ke = use ? min(K, kb + per * KS) : kb;
  if constexpr (std::is_same<TW, double>::value) {
    for (int o = lane; o < NCB * 16 * 16; o += 64) {
      const int c = o >> 4, r = o & 15;
      double acc = 0.0;
      const double* ar = A + (size_t)r * lda;
      for (int k = kb; k < ke; k += 4) {
        const double4 b = bload(c, k);
        acc = fma(ldg<double>(ar + k), b.x, acc);
        acc = fma(ldg<double>(ar + k + 1), b.y, acc);
        acc = fma(ldg<double>(ar + k + 2), b.z, acc);
        acc = fma(ldg<double>(ar + k + 3), b.w, acc);
      }
      red[wave][c][r] = acc;
    }
  } else {
    f32x4 acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    mfma_range<NCB>(A, lda, kb, ke, bload, acc);
    const int rA = lane & 15, g = lane >> 4;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[wave][cb * 16 + rA][4 * g + i] = acc[cb][i];
  }
  __syncthreads();
  for (int p = threadIdx.x; p < IB * NCB * 16 * 16; p += NW * 64) {
    const int slot = p / (NCB * 16 * 16), q = p - slot * (NCB * 16 * 16);
    const int c = q >> 4, r = q & 15;
    T v = red[slot * KSPL][c][r];
#pragma unroll
    for (int w = 1; w < KSPL; ++w) v += red[slot * KSPL + w][c][r];
    S[slot][c][r] = v;
  }
  __syncthreads();
}

// instances per block of a hidden-layer launch.  Stacked instances share the
// weight tile, so a block of ib instances takes less than ib times as long:
// about 1 + 0.6 (ib - 1) blocks' time.  The rule takes the fewest rounds of
// 256 blocks (one per CU) times that length, ties to more stacking.  A
// launch of 384 blocks takes two rounds like one of 512, so the rule follows
// the rounds, not the block count alone.  (The 0.6 is the value that
// reproduces every autotuned choice on the 10k-vertex decoder from 8 to 128
// instances.)
__host__ inline int stack_instances(int row_tiles, int nb, bool f64) {
  if (f64) return 1;
  int best = 1;
  long best_cost = -1;
  for (int ib = 1; ib <= 4; ib *= 2) {
    const long blocks = (long)row_tiles * ((nb + ib - 1) / ib);
    const long cost = ((blocks + 255) / 256) * (5 + 3 * (ib - 1));
    if (best_cost < 0 || cost <= best_cost) {
      best = ib;
      best_cost = cost;
    }
  }
  return best;
}

// ---------------------------------------------------------------------------
// Tall tiles for launches with many instances: one wave per instance slot
// computes MR stacked 16-row tiles x NCB column blocks over the whole K, so
// every B fragment (the instance's activations) serves MR MFMAs and every A
// fragment (the shared weights) NCB.  The operands of the next K-batch are
// loaded before the MFMAs of the current one.  A is [16 MR][lda], K
// contiguous; rows past the layer are never read (16 MR divides m_outp).
// ---------------------------------------------------------------------------
template <int MR, int NCB, typename BL>
__device__ inline void mfma_tall(const float* __restrict__ A, int lda, int K, BL bload, f32x4 (&acc)[MR][NCB]) {
  constexpr int PF = 2;  // K-steps of 16 per batch
  const int lane = threadIdx.x & 63;
  const int rA = lane & 15, g = lane >> 4;
  const float* ap = A + (size_t)rA * lda + 4 * g;
  float4 a0[PF][MR], b0[PF][NCB], a1[PF][MR], b1[PF][NCB];
  // K (a padded width) is a multiple of the batch, so a batch lies wholly
  // inside or past K.  Every batch's loads are issued unconditionally (a
  // batch past K re-reads the last one and is never multiplied): with the
  // same loads on every path the wait before a batch's MFMAs counts only
  // that batch's loads, and the next batch's stay in flight.
  auto load = [&](int k0, float4(&a)[PF][MR], float4(&b)[PF][NCB]) {
    const int kc = min(k0, K - 16 * PF);
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int k = kc + 16 * t;
#pragma unroll
      for (int m = 0; m < MR; ++m) a[t][m] = ldg<float4>(ap + (size_t)16 * m * lda + k);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) b[t][cb] = bload(cb * 16 + rA, k + 4 * g);
    }
  };
  auto mma = [&](const float4(&a)[PF][MR], const float4(&b)[PF][NCB]) {
#pragma unroll
    for (int t = 0; t < PF; ++t)
#pragma unroll
      for (int m = 0; m < MR; ++m)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          acc[m][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][m].x, b[t][cb].x, acc[m][cb], 0, 0, 0);
          acc[m][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][m].y, b[t][cb].y, acc[m][cb], 0, 0, 0);
          acc[m][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][m].z, b[t][cb].z, acc[m][cb], 0, 0, 0);
          acc[m][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][m].w, b[t][cb].w, acc[m][cb], 0, 0, 0);
        }
  };
  // two batches per trip with no branch inside (a load under a branch would
  // be sunk to its use); an odd last batch is already in a0 after the loop.
  // The scheduling barriers keep each batch's loads ahead of the MFMAs of
  // the batch before it.
  constexpr int KB = 16 * PF;
  const int nbat = K / KB;
  load(0, a0, b0);
  int i = 0;
  for (; i + 1 < nbat; i += 2) {
    load((i + 1) * KB, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    mma(a0, b0);
    load((i + 2) * KB, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    mma(a1, b1);
  }
  if (i < nbat) mma(a0, b0);
}

template <int MR, int NCB, typename BL>
__device__ inline void mfma_tall(const __bf16* __restrict__ A, int lda, int K, BL bload, f32x4 (&acc)[MR][NCB]) {
  const int lane = threadIdx.x & 63;
  const int rA = lane & 15, g = lane >> 4;
  const __bf16* ap = A + (size_t)rA * lda + 8 * g;
  bf16x8 a0[MR], a1[MR];
  bf16x8 b0[NCB], b1[NCB];
  // unconditional loads of whole K-steps, as in the FP32 form
  auto load = [&](int k, bf16x8(&a)[MR], bf16x8(&b)[NCB]) {
    const int kc = min(k, K - 32);
#pragma unroll
    for (int m = 0; m < MR; ++m) a[m] = ldg<bf16x8>(ap + (size_t)16 * m * lda + kc);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) b[cb] = bfrag(bload, cb * 16 + rA, kc + 8 * g);
  };
  auto mma = [&](const bf16x8(&a)[MR], const bf16x8(&b)[NCB]) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int m = 0; m < MR; ++m) acc[m][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[cb], acc[m][cb], 0, 0, 0);
  };
  const int nbat = K / 32;
  load(0, a0, b0);
  int i = 0;
  for (; i + 1 < nbat; i += 2) {
    load((i + 1) * 32, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    mma(a0, b0);
    load((i + 2) * 32, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    mma(a1, b1);
  }
  if (i < nbat) mma(a0, b0);
}

// Tall tile of every instance slot (waves KS s .. KS s + KS - 1 = slot s,
// wave h of a slot taking the h-th part of K in 32-wide steps) into
// S[slot][c][r], r < 16 MR, the parts added in order; a slot not in use
// writes zeros.  Ends with a barrier.
template <typename TW, int NCB, int MR, int KS, typename BL>
__device__ inline void gemm_tall(const TW* __restrict__ A, int lda, int K, bool use, BL bload,
                                 float (*S)[NCB * 16][16 * MR + 1]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = wave / KS, part = wave - slot * KS;
  const int nst = K / 32;
  const int k0 = 32 * ((nst * part) / KS), k1 = 32 * ((nst * (part + 1)) / KS);
  f32x4 acc[MR][NCB];
#pragma unroll
  for (int m = 0; m < MR; ++m)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[m][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (use && k1 > k0) {
    auto bpart = [&](int c, int k) { return bload(c, k0 + k); };
    mfma_tall<MR, NCB>(A + k0, lda, k1 - k0, bpart, acc);
  }
  const int rA = lane & 15, g = lane >> 4;
#pragma unroll
  for (int h = 0; h < KS; ++h) {
    if (part == h)
#pragma unroll
      for (int m = 0; m < MR; ++m)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float& d = S[slot][cb * 16 + rA][16 * m + 4 * g + i];
            d = (h == 0 ? 0.f : d) + acc[m][cb][i];
          }
    __syncthreads();
  }
}

// LDS staging of the tall tiles.  Read straight from global memory, an MFMA
// operand fragment puts the 16 lanes of each quarter-wave on 16 different
// rows, so every lane's 16 bytes are a request of their own and the address
// unit takes about a cycle per lane: in BF16 it, not the MFMAs, bounds a
// wave, and in FP32 it takes about as long as the MFMAs.  Here the block
// copies each K-chunk of the weight tile (which its instance slots share)
// and of every slot's B tile into LDS with loads in which consecutive lanes
// read consecutive 16 bytes, and the waves read their fragments from LDS
// rows padded by 16 bytes, which puts the 16 rows of a quarter-wave's reads
// on disjoint banks.  A sub-chunk is 64 bytes of a row (32 BF16 or 16 FP32
// K entries: one BF16 MFMA step, four FP32 ones); a chunk is KS sub-chunks,
// which the KS waves of a slot take in turn.  Two LDS buffers, and register
// sets that load chunks ahead of the one being multiplied.
#ifndef TALL_CHUNKS_IN_FLIGHT
#define TALL_CHUNKS_IN_FLIGHT 2
#endif
template <typename TW, int NCB, int MR, int IB, int KS>
struct tall_stage {
  static constexpr int SW = 64 / (int)sizeof(TW);  // K entries of a sub-chunk
  static constexpr int KC = SW * KS;              // K per chunk
  static constexpr int LD = 64 * KS + 16;         // bytes per staged row
  static constexpr int AROWS = 16 * MR, BROWS = IB * NCB * 16;
  static constexpr int BYTES = 2 * (AROWS + BROWS) * LD;
  // two waves per slot, within about a third of the 160 KB of LDS beside
  // the epilogue's
  static constexpr bool on = (std::is_same<TW, __bf16>::value || std::is_same<TW, float>::value) && MR > 1 &&
                             KS == 2 && BYTES <= 96 * 1024;
};

// K-split of the tall tiles: waves per instance slot.  With one block per CU
// a single wave per SIMD leaves the MFMAs idle through every wait for LDS
// and every barrier, so two waves per slot take alternate parts of K.  A
// BF16 wave's MFMAs take a sixteenth of an FP32 wave's time, so BF16 splits
// K in the direct form too; FP32 splits only the staged form (a direct
// FP32 tile with 128 jet columns was slower split).
template <typename TW, int NCB, int MR>
struct tall_ks {
  static constexpr int v = std::is_same<TW, __bf16>::value || tall_stage<TW, NCB, MR, 4, 2>::on ? 2 : 1;
};

// B is the slot's operand, column c at B + c ldb (K contiguous), in the
// weights' type.
template <typename TW, int NCB, int MR, int IB, int KS>
__device__ inline void gemm_tall_lds(const TW* __restrict__ A, int lda, int K, bool use, const TW* __restrict__ B,
                                     int ldb, float (*S)[NCB * 16][16 * MR + 1], unsigned char* stage) {
  using G = tall_stage<TW, NCB, MR, IB, KS>;
  typedef typename std::conditional<std::is_same<TW, float>::value, float4, bf16x8>::type P;  // 16 bytes
  constexpr int PE = 16 / (int)sizeof(TW);  // K entries of a piece
  constexpr int NT = 64 * IB * KS, NG = 64 * KS;
  constexpr int PR = G::KC / PE;  // 16-byte pieces of a staged row
  constexpr int NA = G::AROWS * PR;
  constexpr int PA = (NA + NT - 1) / NT, PB = NCB * 16 * PR / NG;
  constexpr int D = TALL_CHUNKS_IN_FLIGHT;  // register sets: chunks loaded ahead
  static_assert(NCB * 16 * PR % NG == 0, "B pieces split evenly over a slot's threads");
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int slot = wave / KS, part = wave - slot * KS, tg = tid - slot * NG;
  const int nch = (K + G::KC - 1) / G::KC;
  // chunk ch into registers, nothing applied to the loaded values (an
  // operation on them would wait for the load right there).  Pieces past K
  // (the second half of a last chunk) are loaded from a clamped index and
  // never multiplied: K is a multiple of 32, so a wave's sub-chunk lies
  // wholly inside or past K.  A slot not in use loads the same number of
  // pieces, from the weight tile: its table entry may be an empty pool
  // slot's, whose pointers are null or stale.
  const TW* Bs = use ? B : A;
  const int lds_b = use ? ldb : lda, cmod = use ? NCB * 16 : G::AROWS;
  auto gload = [&](int ch, P(&ra)[PA], P(&rb)[PB]) {
    const int k0 = ch * G::KC;
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      const int q = min(tid + i * NT, NA - 1);
      ra[i] = ldg<P>(A + (size_t)(q / PR) * lda + min(k0 + PE * (q % PR), K - PE));
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int q = tg + i * NG;
      rb[i] = ldg<P>(Bs + (size_t)((q / PR) % cmod) * lds_b + min(k0 + PE * (q % PR), K - PE));
    }
  };
  auto lstore = [&](int buf, const P(&ra)[PA], const P(&rb)[PB]) {
    unsigned char* base = stage + buf * (G::AROWS + G::BROWS) * G::LD;
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      const int q = tid + i * NT;
      if (q < NA) *reinterpret_cast<P*>(base + (q / PR) * G::LD + 16 * (q % PR)) = ra[i];
    }
    unsigned char* bb = base + (G::AROWS + slot * NCB * 16) * G::LD;
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int q = tg + i * NG;
      *reinterpret_cast<P*>(bb + (q / PR) * G::LD + 16 * (q % PR)) = rb[i];
    }
  };
  f32x4 acc[MR][NCB];
#pragma unroll
  for (int m = 0; m < MR; ++m)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[m][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int rA = lane & 15, g = lane >> 4;
  // this wave's 32-wide sub-chunk of chunk ch, from LDS buffer ch & 1
  // (lane group g holds the sub-chunk's g-th 16 bytes of its row: BF16 one
  // 32-deep MFMA step; FP32 four 4-deep ones, entry j of every group in step j)
  auto mma = [&](int ch) {
    const int kk = ch * G::KC + G::SW * part;
    if (use && kk < K) {  // uniform over the wave
      const unsigned char* base = stage + (ch & 1) * (G::AROWS + G::BROWS) * G::LD + 64 * part + 16 * g;
      const unsigned char* bb = base + (G::AROWS + slot * NCB * 16) * G::LD;
      P a[MR], b[NCB];
#pragma unroll
      for (int m = 0; m < MR; ++m) a[m] = *reinterpret_cast<const P*>(base + (16 * m + rA) * G::LD);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) b[cb] = *reinterpret_cast<const P*>(bb + (16 * cb + rA) * G::LD);
      if constexpr (std::is_same<TW, float>::value) {
        // the MR NCB independent tiles between two steps on one accumulator
        auto step = [&](auto pick) {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int m = 0; m < MR; ++m)
              acc[m][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(pick(a[m]), pick(b[cb]), acc[m][cb], 0, 0, 0);
        };
        step([](const float4& v) { return v.x; });
        step([](const float4& v) { return v.y; });
        step([](const float4& v) { return v.z; });
        step([](const float4& v) { return v.w; });
      } else {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int m = 0; m < MR; ++m) acc[m][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[cb], acc[m][cb], 0, 0, 0);
      }
    }
  };
  // register set d holds chunk ch = d (mod D).  Step ch: refill set d with
  // chunk ch + D (chunk ch is in LDS already), multiply chunk ch, store
  // chunk ch + 1 into the other LDS buffer, barrier.  A chunk's loads have
  // D - 1 steps to land before its LDS store waits for them.  No load sits
  // under a branch, so that each wait counts only the loads it needs: the
  // steps run in whole rounds of D, loads past the last chunk re-read it
  // (clamped), and steps past it multiply nothing.
  const int nst = (nch + D - 1) / D * D;
  P ra[D][PA], rb[D][PB];
#pragma unroll
  for (int d = 0; d < D; ++d) gload(min(d, nch - 1), ra[d], rb[d]);
  lstore(0, ra[0], rb[0]);
  __syncthreads();
  for (int ch0 = 0; ch0 < nst; ch0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int ch = ch0 + d;
      gload(min(ch + D, nch - 1), ra[d], rb[d]);
      mma(ch);
      lstore((ch + 1) & 1, ra[(d + 1) % D], rb[(d + 1) % D]);
      __syncthreads();
    }
  }
  // S may share the staging buffers: every wave has passed the last barrier
#pragma unroll
  for (int h = 0; h < KS; ++h) {
    if (part == h)
#pragma unroll
      for (int m = 0; m < MR; ++m)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float& d = S[slot][cb * 16 + rA][16 * m + 4 * g + i];
            d = (h == 0 ? 0.f : d) + acc[m][cb][i];
          }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Forward hidden layer l with the jet activation.  One block per 16 MR rows.
// ---------------------------------------------------------------------------
// Input k of stencil column c of the central differences (the column order
// of the last hidden layer's stencils; zero past the 14 n_q + 3 columns).
template <typename T>
__device__ inline T fd_input(int c, int k, int nq, T q, T dq, T qd, T h) {
  if (c == 0) return q;
  if (c < 1 + 2 * nq) {
    const int idx = c - 1, j = idx >> 1;
    return q + ((k == j) ? ((idx & 1) ? -h : h) : T(0));
  }
  if (c < 1 + 14 * nq) {
    const int idx = c - 1 - 2 * nq, blk = idx / (4 * nq), rem = idx - blk * 4 * nq;
    const int j = rem >> 2, sub = rem & 3;
    const T e = (k == j) ? ((sub & 1) ? -h : h) : T(0);
    const T v = (blk == 1 ? h * qd : blk == 2 ? T(2) * h * dq : h * dq);
    return (q + e) + ((sub & 2) ? -v : v);
  }
  if (c < 3 + 14 * nq) {
    const T v = T(2) * h * dq;
    return (c == 1 + 14 * nq) ? q + v : q - v;
  }
  return T(0);
}

// JG > 0: jet groups.  A block computes the four base channels and the four
// channels of JG perturbations e_j (16 columns for JG = 3), so the columns
// of one row tile spread over ceil(n_q / JG) blocks (blockIdx.y = instance x
// groups + group), each splitting K over eight waves.  Where the whole-tile
// form does the same (at most four column blocks) every column is the same
// K sum, so the results are the same bits.  The base channels, which every
// group needs for its activation derivatives, are stored by group 0 only.
template <typename T, typename TW, int NCB, int IB, bool FD, int MR, int JG = 0>
__global__ __launch_bounds__(MR > 1 ? 64 * IB * (tall_ks<TW, NCB, MR>::v) : 512) void k_fwd_hidden(LayerArgs la,
                                                                                       const Inst<T>* __restrict__ tab,
                                                                                       int nb) {
  static_assert(MR == 1 || (!FD && std::is_same<T, float>::value), "tall tiles: complex-step FP32 jets only");
  static_assert(JG == 0 || (NCB == 1 && IB == 1 && MR == 1 && !FD && 4 + 4 * JG == 16), "jet groups: one column block");
  constexpr int ROWS = 16 * MR;  // output rows of a block
  constexpr int NW = MR > 1 ? IB * tall_ks<TW, NCB, MR>::v : splitk_waves<T, NCB>::v;
  constexpr int KSPL = NW / IB;
  constexpr int NG = KSPL * 64;  // threads of one instance slot
  const int l = la.l;
  const int tid = threadIdx.x, wave = tid >> 6;
  const int slot = wave / KSPL, tg = tid - slot * NG;
  // several instances: each XCD takes whole instance groups, whose
  // activations every row tile reads, so they stay in one L2
  int bx = blockIdx.x, by = blockIdx.y;
  if (!JG && gridDim.y > 1) xcd_block(bx, by);
  const int ngrp = JG ? gridDim.y / nb : 1;
  const int inst = JG ? by / ngrp : by * IB + slot;
  const int grp = JG ? by - inst * ngrp : 0;
  const Inst<T>& I = tab[min(inst, nb - 1)];
  // the table entry's fields are read before any test so that their scalar
  // loads leave together
  constexpr bool fd = FD;  // central differences instead of complex-step jets
  const int active = I.active, nq = I.n_q, trimmed = I.trimmed;
  const T* X = (l & 1) ? I.act0 : I.act1;
  T* const outp = (l & 1) ? I.act1 : I.act0;
  T* const pre = I.pre[l];
  T* const fold = I.fold;
  const double* din = I.dec_in;
  const double dt64 = I.dt, fdh64 = I.fd_h;
  const int m_inp = la.m_inp, m_out = la.m_out, m_outp = la.m_outp;
  load_now(active, nq, trimmed, X, outp, pre, fold, din, dt64, fdh64, m_inp, m_out, m_outp, la.W, la.b, la.act, la.L);
  const bool use = inst < nb && active;
  const T dtT = (T)dt64;
  const int row0 = bx * ROWS;
  if (row0 >= m_outp || (IB == 1 && !use)) return;  // uniform over the block
  const TW* W = reinterpret_cast<const TW*>(la.W) + (size_t)row0 * m_inp;
  const T* bias = reinterpret_cast<const T*>(la.b);
  using STG = tall_stage<TW, NCB, MR, IB, tall_ks<TW, NCB, MR>::v>;
  constexpr int SB = (int)sizeof(T) * IB * NCB * 16 * (ROWS + 1), GB = STG::on ? STG::BYTES : 0;
  __shared__ __align__(16) unsigned char lds_s[SB > GB ? SB : GB];  // S, or the GEMM's staging before it
  T(*S)[NCB * 16][ROWS + 1] = reinterpret_cast<T(*)[NCB * 16][ROWS + 1]>(lds_s);
  __shared__ T red[MR == 1 ? NW : 1][NCB * 16][16];
  __shared__ T sd1[IB][ROWS], sd2[IB][ROWS], sd3[IB][ROWS], sx2[IB][ROWS], sx4[IB][ROWS], sx23[IB][ROWS];
  typedef typename vec4<T>::type V4;

  // the bias of this tile is loaded before the GEMM (no dependent round trip)
  const T bias_v = (tg < ROWS && row0 + tg < m_out) ? ldg<T>(bias + row0 + tg) : T(0);
  // B operands: the input jets (layer 0, formed from the decoder input) or
  // the previous layer's jets.  The GEMM is instantiated once for each, so
  // that its K loop has the same loads on every path.
  auto bload_in = [&](int c, int k) -> V4 {
    if constexpr (FD) {
      // stencil columns of the central differences: q, q +- h e_j, then per j
      // q +- h e_j +- v for v = h dq, h qdot, 2h dq, then q +- 2h dq; every
      // input formed in T (loads from clamped indices, then selects)
      T v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int kk = min(k + t, nq - 1);
        const T q = (T)ldg<double>(din + kk), dq = (T)ldg<double>(din + nq + kk);
        const T qd = (T)ldg<double>(din + 2 * nq + kk);
        v[t] = fd_input<T>(c, kk, nq, q, dq, qd, (T)fdh64);
        v[t] = (k + t < nq) ? v[t] : T(0);
      }
      return V4{v[0], v[1], v[2], v[3]};
    }
    // input jets: value q, tangents dq (i2) and qdot (i4), unit e_j (i1);
    // loads from clamped indices, then selects (no load under a branch)
    const int ch = min(c, 2);
    T v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int kk = k + t;
      const T x = (T)ldg<double>(din + ch * nq + min(kk, nq - 1));
      T y = (c < 3) ? x : (c >= 4 && c - 4 == kk) ? T(1) : T(0);
      v[t] = (kk < nq && c < 4 + nq) ? y : T(0);
    }
    return V4{v[0], v[1], v[2], v[3]};
  };
  // a BF16 decoder's hidden activations are stored as BF16 (the MFMA operand
  // they become); complex-step jets only
  constexpr bool BFX = std::is_same<TW, __bf16>::value && !FD;
  auto bload_x = [&](int c, int k) {
    if constexpr (BFX) return ldg<bf16x8>(reinterpret_cast<const __bf16*>(X) + (size_t)c * m_inp + k);
    else return ldg<V4>(X + (size_t)c * m_inp + k);
  };
  // jet channel of local column c of a jet group (-1: past n_q)
  auto gcol = [&](int c) -> int {
    if (c < 4) return c;
    constexpr int jg = JG > 0 ? JG : 1;
    const int role = (c - 4) / jg, j = grp * jg + (c - 4 - role * jg);
    return j < nq ? 4 + role * nq + j : -1;
  };
  auto gemm = [&](auto bload, auto x_operand) {
    if constexpr (JG > 0) {
      auto bload_g = [&](int c, int k) {
        const int gc = gcol(c);
        const auto v = bload(max(gc, 0), k);
        return gc >= 0 ? v : zero_of<std::remove_const_t<decltype(v)>>();
      };
      gemm_splitk<T, TW, NCB, NW, IB>(W, m_inp, m_inp, use, bload_g, S, red);
    } else if constexpr (MR == 1) gemm_splitk<T, TW, NCB, NW, IB>(W, m_inp, m_inp, use, bload, S, red);
    else if constexpr (STG::on && decltype(x_operand)::value)  // the previous layer's activations, stored as TW
      gemm_tall_lds<TW, NCB, MR, IB, tall_ks<TW, NCB, MR>::v>(W, m_inp, m_inp, use, reinterpret_cast<const TW*>(X), m_inp, S,
                                                     lds_s);
    else gemm_tall<TW, NCB, MR, tall_ks<TW, NCB, MR>::v>(W, m_inp, m_inp, use, bload, S);
  };
  if (l == 0) gemm(bload_in, std::false_type());  // uniform over the block
  else gemm(bload_x, std::true_type());

  T(*Ss)[ROWS + 1] = S[slot];
  if constexpr (FD) {
    // central differences: every column is a forward pass of its own (bias
    // and activation on each); the base and q +- h e_j keep their
    // pre-activations for backpropagation.  fd is the same for every slot.
    __shared__ T sbias[IB][16];
    if (use && tg < 16) sbias[slot][tg] = bias_v;
    __syncthreads();
    if (use) {
      const int C = 14 * nq + 3;
      for (int p = tg; p < 16 * C; p += NG) {
        const int r = p & 15, c = p >> 4;
        const bool valid = row0 + r < m_out;
        const T x = Ss[c][r] + sbias[slot][r];
        T y, d1, d2, d3;
        act_jet(la.act, x, y, d1, d2, d3);
        if (c < 1 + 2 * nq) stg<T>(pre + (size_t)c * m_outp + row0 + r, valid ? x : T(0));
        Ss[c][r] = valid ? y : T(0);
      }
    }
    __syncthreads();
  } else {
  if (use && tg < ROWS) {
    const int row = row0 + tg;
    const bool valid = row < m_out;
    const T x0 = Ss[0][tg] + bias_v;
    const T x2 = Ss[1][tg], x4 = Ss[2][tg], x23 = Ss[3][tg];
    T y, d1, d2, d3;
    act_jet(la.act, x0, y, d1, d2, d3);
    sd1[slot][tg] = d1; sd2[slot][tg] = d2; sd3[slot][tg] = d3;
    sx2[slot][tg] = x2; sx4[slot][tg] = x4; sx23[slot][tg] = x23;
    if (grp == 0) stg<T>(pre + row, valid ? x0 : T(0));
    Ss[0][tg] = valid ? y : T(0);
    Ss[1][tg] = valid ? d1 * x2 : T(0);
    Ss[2][tg] = valid ? d1 * x4 : T(0);
    Ss[3][tg] = valid ? d1 * x23 + d2 * x2 * x2 : T(0);
  }
  __syncthreads();
  if (use) {
    // the jets of perturbation j sit in local columns 4 + jl + {0,1,2,3} nl
    const int nl = JG ? JG : nq;
    for (int p = tg; p < ROWS * nl; p += NG) {
      const int r = p & (ROWS - 1), jl = p / ROWS, j = grp * JG + jl;
      if (JG && j >= nq) continue;
      const bool valid = row0 + r < m_out;
      const T x1 = Ss[4 + jl][r], x12 = Ss[4 + nl + jl][r], x14 = Ss[4 + 2 * nl + jl][r], x123 = Ss[4 + 3 * nl + jl][r];
      const T d1 = sd1[slot][r], d2 = sd2[slot][r], d3 = sd3[slot][r];
      const T x2 = sx2[slot][r], x4 = sx4[slot][r], x23 = sx23[slot][r];
      stg<T>(pre + (size_t)(1 + j) * m_outp + row0 + r, valid ? x1 : T(0));
      Ss[4 + jl][r] = valid ? d1 * x1 : T(0);
      Ss[4 + nl + jl][r] = valid ? d1 * x12 + d2 * x1 * x2 : T(0);
      Ss[4 + 2 * nl + jl][r] = valid ? d1 * x14 + d2 * x1 * x4 : T(0);
      Ss[4 + 3 * nl + jl][r] = valid ? d1 * x123 + d2 * (x1 * x23 + T(2) * x2 * x12) + d3 * x1 * x2 * x2 : T(0);
    }
  }
  __syncthreads();
  }
  if (!use) return;
  if (l + 2 < la.L) {
    if constexpr (JG > 0) {
      for (int p = tg; p < 16 * 16; p += NG) {
        const int c = p >> 4, r = p & 15, gc = gcol(c);
        if (gc >= 0 && (c >= 4 || grp == 0)) {
          if constexpr (BFX) stg<__bf16>(reinterpret_cast<__bf16*>(outp) + (size_t)gc * m_outp + row0 + r, (__bf16)Ss[c][r]);
          else stg<T>(outp + (size_t)gc * m_outp + row0 + r, Ss[c][r]);
        }
      }
      return;
    }
    // tall tiles: 8 BF16 or 4 FP32 rows of a column per store (with 16-row
    // tiles the wider items leave too many threads idle)
    const int C = fd ? 14 * nq + 3 : 4 + 4 * nq;
    constexpr int VG = MR == 1 ? 1 : BFX ? 8 : 4, RG = ROWS / VG;
    for (int p = tg; p < C * RG; p += NG) {
      const int c = p / RG, r = VG * (p - c * RG);
      if constexpr (VG == 1) {
        if constexpr (BFX) stg<__bf16>(reinterpret_cast<__bf16*>(outp) + (size_t)c * m_outp + row0 + r, (__bf16)Ss[c][r]);
        else stg<T>(outp + (size_t)c * m_outp + row0 + r, Ss[c][r]);
      } else if constexpr (BFX) {
        bf16x8 o;
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = (__bf16)Ss[c][r + i];
        stg<bf16x8>(reinterpret_cast<__bf16*>(outp) + (size_t)c * m_outp + row0 + r, o);
      } else {
        stg<V4>(outp + (size_t)c * m_outp + row0 + r, V4{Ss[c][r], Ss[c][r + 1], Ss[c][r + 2], Ss[c][r + 3]});
      }
    }
  } else {
    // last hidden layer: fold into the output channels (the output layer is
    // linear, so eq. delta_j can be combined before it); the trimmed
    // formulation keeps H.(dq - dt qdot) and no H(dq, dq)
    const T dt = dtT;
    const int C = 2 + 2 * nq;
    if constexpr (FD) {
      // the stencils of the central differences (as in the FP64 oracle's
      // order of operations); the trimmed formulation as above
      const T h = (T)fdh64, h2 = T(2) * h, h4 = T(4) * h * h;
      const int base = 1 + 2 * nq;
      for (int p = tg; p < C * 16; p += NG) {
        const int c = p >> 4, r = p & 15;
        T v;
        if (c == 0) v = Ss[0][r];
        else if (c <= nq) {
          const int j = c - 1;
          v = (Ss[1 + 2 * j][r] - Ss[2 + 2 * j][r]) / h2;
        } else if (c <= 2 * nq) {
          const int j = c - 1 - nq;
          const int b0 = base + 4 * j, b1 = base + 4 * (nq + j), b2 = base + 4 * (2 * nq + j);
          const T Hdq = (Ss[b0][r] - Ss[b0 + 1][r] - Ss[b0 + 2][r] + Ss[b0 + 3][r]) / h4;
          const T Hv = (Ss[b1][r] - Ss[b1 + 1][r] - Ss[b1 + 2][r] + Ss[b1 + 3][r]) / h4;
          const T gp = (Ss[b2][r] - T(2) * Ss[1 + 2 * j][r] + Ss[b2 + 2][r]) / h4;
          const T gm = (Ss[b2 + 1][r] - T(2) * Ss[2 + 2 * j][r] + Ss[b2 + 3][r]) / h4;
          const T Sdd = (gp - gm) / h2;
          v = trimmed ? Hdq - dt * Hv : Sdd + T(3) * Hdq - dt * Hv;
        } else {
          v = trimmed ? T(0) : (Ss[base + 12 * nq][r] - T(2) * Ss[0][r] + Ss[base + 12 * nq + 1][r]) / h4;
        }
        stg<T>(fold + (size_t)c * m_outp + row0 + r, v);
      }
      return;
    }
    if constexpr (JG > 0) {
      // fold entry f of a group: 0 the value and 1 the (dq, dq) channel
      // (group 0), then J and dJ of the group's perturbations
      for (int p = tg; p < (2 + 2 * JG) * 16; p += NG) {
        const int f = p >> 4, r = p & 15;
        const int jl = (f - 2) % JG, j = grp * JG + jl;
        if (f < 2 ? grp != 0 : j >= nq) continue;
        T v;
        int c;
        if (f == 0) {
          c = 0;
          v = Ss[0][r];
        } else if (f == 1) {
          c = 1 + 2 * nq;
          v = trimmed ? T(0) : Ss[3][r];
        } else if (f < 2 + JG) {
          c = 1 + j;
          v = Ss[4 + jl][r];
        } else {
          c = 1 + nq + j;
          v = trimmed ? Ss[4 + JG + jl][r] - dt * Ss[4 + 2 * JG + jl][r]
                      : Ss[4 + 3 * JG + jl][r] + T(3) * Ss[4 + JG + jl][r] - dt * Ss[4 + 2 * JG + jl][r];
        }
        stg<T>(fold + (size_t)c * m_outp + row0 + r, v);
      }
      return;
    }
    for (int p = tg; p < C * ROWS; p += NG) {
      const int c = p / ROWS, r = p & (ROWS - 1);
      T v;
      if (c == 0) v = Ss[0][r];
      else if (c <= nq) v = Ss[4 + c - 1][r];
      else if (c <= 2 * nq) {
        const int j = c - 1 - nq;
        v = trimmed ? Ss[4 + nq + j][r] - dt * Ss[4 + 2 * nq + j][r]
                    : Ss[4 + 3 * nq + j][r] + T(3) * Ss[4 + nq + j][r] - dt * Ss[4 + 2 * nq + j][r];
      } else v = trimmed ? T(0) : Ss[3][r];
      stg<T>(fold + (size_t)c * m_outp + row0 + r, v);
    }
  }
}

// ---------------------------------------------------------------------------
// Output layer: rec[i][c] = keep_i (W_L fold + b_L e_0)[i][c] for the decoded
// rows (all N, or the DOFs of cubature tets on the Gram path).  One block per
// 16-row tile; its OUT_SPLIT waves each take a quarter of K, holding their
// weight and folded-activation operands in registers, and the partial tiles
// are added in LDS in wave order.  The row ids are read first, then weights,
// bias and mask of those rows together with the folded activations.
// ---------------------------------------------------------------------------
#define OUT_SPLIT 4
#define OUT_KMAX 256  // last hidden layer: K <= 256


template <typename TW, int NCB>
__global__ __launch_bounds__(64 * OUT_SPLIT) void k_fwd_out(LayerArgs la, const Inst<float>* __restrict__ tab) {
  const Inst<float>& I = tab[blockIdx.y];
  const int inst_active = I.active, gram = I.gram, n_cd = I.n_cdofs, N = I.N, Cf = I.Cf;
  const int* cdofs = I.cdofs;
  const float* fold = I.fold;
  float* rec = I.rec;
  const float* keep = I.keep;
  const int K = la.m_inp;
  load_now(inst_active, gram, n_cd, N, Cf, cdofs, fold, rec, keep, K, la.W, la.b);
  const int nrows = gram ? n_cd : N;
  const int row0 = blockIdx.x * 16;
  if (!inst_active || row0 >= nrows) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rA = lane & 15, g = lane >> 4;
  const TW* W = reinterpret_cast<const TW*>(la.W);
  const float* bias = reinterpret_cast<const float*>(la.b);
  constexpr int KS = kstep<TW>::v;
  constexpr int NT = (OUT_KMAX / OUT_SPLIT + KS - 1) / KS;  // K-steps of one wave
  const int kq = K / OUT_SPLIT, kb = wave * kq, ke = kb + kq;
  __shared__ float red[OUT_SPLIT][NCB * 16][17];
  __shared__ int srow[16];
  __shared__ float sbias[16], skeep[16];
  // 1) row ids: the weight row of this lane (direct path: rows past N are the
  //    zero padding of W_L; Gram path: the last listed row) and, for threads
  //    0..15, the output row of the epilogue; folded activations meanwhile
  const int wrow = gram ? ldg<int>(cdofs + min(row0 + rA, nrows - 1)) : row0 + rA;
  const int tr = min(row0 + (int)(threadIdx.x & 15), nrows - 1);
  const int orow = gram ? ldg<int>(cdofs + tr) : tr;
  typedef typename std::conditional<std::is_same<TW, float>::value, float4, bf16x8>::type AF;
  float4 bf[NT][NCB][KS / 16];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int h = 0; h < KS / 16; ++h) {
        const int k = min(kb + t * KS + (KS / 4) * g + 4 * h, K - 4);
        bf[t][cb][h] = ldg<float4>(fold + (size_t)(cb * 16 + rA) * K + k);
      }
  // 2) weights of this lane's row, bias and mask of the output rows
  // a lane group whose K entries start past this wave's quarter (K < 256)
  // contributes a zero A operand; its load is from a clamped address
  AF a[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int kk = kb + t * KS + (KS / 4) * g;
    const AF v = ldg<AF>(W + (size_t)wrow * K + min(kk, K - KS / 4));
    a[t] = kk < ke ? v : zero_of<AF>();
  }
  if (threadIdx.x < 16) {
    srow[threadIdx.x] = orow;
    sbias[threadIdx.x] = ldg<float>(bias + orow);
    skeep[threadIdx.x] = ldg<float>(keep + orow);
  }
  f32x4 acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (kb + t * KS < ke) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        if constexpr (std::is_same<TW, float>::value) {
          const float4 b = bf[t][cb][0];
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t].x, b.x, acc[cb], 0, 0, 0);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t].y, b.y, acc[cb], 0, 0, 0);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t].z, b.z, acc[cb], 0, 0, 0);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t].w, b.w, acc[cb], 0, 0, 0);
        } else {
          const bf16x8 b = to_bf16x8(bf[t][cb][0], bf[t][cb][KS / 16 - 1]);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], b, acc[cb], 0, 0, 0);
        }
      }
    }
  }
  // partial tiles: item i of lane l is D[4 (l/16) + i][l % 16]
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wave][cb * 16 + rA][4 * g + i] = acc[cb][i];
  __syncthreads();
  // the launch may decode fewer channels than the record holds (the Gram
  // path needs the value and J only)
  const int nc = min(Cf, NCB * 16);
  for (int p = threadIdx.x; p < 16 * nc; p += 64 * OUT_SPLIT) {
    const int c = p >> 4, r = p & 15;
    if (row0 + r < nrows) {
      float v = red[0][c][r];
#pragma unroll
      for (int w = 1; w < OUT_SPLIT; ++w) v += red[w][c][r];
      if (c == 0) v += sbias[r];
      stg<float>(rec + (size_t)srow[r] * Cf + c, v * skeep[r]);
    }
  }
}

// Output layer for many instances: a block of OUT_SPLIT waves stages the
// folded activations [Cf][K] of NI instances in LDS once and each wave takes
// OUT_TILES 16-row tiles over the whole K, the weights of its next tile loaded
// while the MFMAs of the current one run.  NI = 2 when every instance of the
// launch decodes the same rows (the same cubature DOFs, or all N rows of equal
// N): the two instances of a block then share each weight fragment.  The K
// quarters of the split kernel above are kept as four accumulators and added
// in the same order, so both kernels give the same bits.
#define OUT_TILES 2
template <typename TW, int NCB, int NI>
__global__ __launch_bounds__(64 * OUT_SPLIT) void k_fwd_out_wide(LayerArgs la, const Inst<float>* __restrict__ tab,
                                                                 int nb, const int* __restrict__ rows) {
  const int i0 = blockIdx.y * NI;
  const Inst<float>& I = tab[i0];
  const Inst<float>& I1 = tab[min(i0 + NI - 1, nb - 1)];  // the second instance (NI = 2)
  // The row set and sizes come from an instance in use (the entry of an
  // empty pool slot may be zero or left by a destroyed instance: its
  // pointers are never followed); a pool passes its own copy of the rows.
  const Inst<float>& Ir = (NI == 1 || I.active) ? I : I1;
  const int act0 = I.active, act1 = I1.active, gram = Ir.gram, n_cd = Ir.n_cdofs, N = Ir.N, Cf = Ir.Cf;
  const int* cdofs = rows ? rows : Ir.cdofs;
  const float* fold0 = I.fold;
  const float* fold1 = I1.fold;
  float* rec0 = I.rec;
  float* rec1 = I1.rec;
  const float* keep0 = I.keep;
  const float* keep1 = I1.keep;
  const int K = la.m_inp;
  load_now(act0, act1, gram, n_cd, N, Cf, cdofs, fold0, fold1, rec0, rec1, keep0, keep1, K, la.W, la.b);
  bool use[NI];
  use[0] = act0 != 0;
  if constexpr (NI > 1) use[1] = act1 != 0 && i0 + 1 < nb;
  const int nrows = gram ? n_cd : N;
  constexpr int BROWS = 16 * OUT_SPLIT * OUT_TILES;
  const int blk0 = blockIdx.x * BROWS;
  bool any = use[0];
  if constexpr (NI > 1) any = any || use[1];
  if (!any || blk0 >= nrows) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rA = lane & 15, g = lane >> 4;
  const TW* W = reinterpret_cast<const TW*>(la.W);
  const float* bias = reinterpret_cast<const float*>(la.b);
  constexpr int KS = kstep<TW>::v;
  constexpr int NT = (OUT_KMAX / OUT_SPLIT + KS - 1) / KS;  // K-steps of one quarter
  const int kq = K / OUT_SPLIT;
  typedef typename std::conditional<std::is_same<TW, float>::value, float4, bf16x8>::type AF;
  __shared__ __align__(16) float Fs[NI][NCB * 16][OUT_KMAX + 4];
  // the folded activations, coalesced, once per block: every load of an
  // instance is issued (from clamped indices) before its LDS writes.  An
  // instance not in use leaves its copy unwritten; its results are never
  // stored.
  auto stage_fold = [&]() {
    constexpr int FI = NCB * 16 * (OUT_KMAX / 4) / (64 * OUT_SPLIT);  // float4 items per thread at K = OUT_KMAX
    const int nk4 = K / 4, nit = NCB * 16 * nk4;
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      if (!use[j]) continue;
      const float* fold = j == 0 ? fold0 : fold1;
      float4 v[FI];
#pragma unroll
      for (int it = 0; it < FI; ++it) {
        const int p = min((int)threadIdx.x + it * 64 * OUT_SPLIT, nit - 1), c = p / nk4;
        v[it] = ldg<float4>(fold + (size_t)c * K + 4 * (p - c * nk4));
      }
#pragma unroll
      for (int it = 0; it < FI; ++it) {
        const int p = (int)threadIdx.x + it * 64 * OUT_SPLIT, c = p / nk4;
        if (p < nit) *reinterpret_cast<float4*>(&Fs[j][c][4 * (p - c * nk4)]) = v[it];
      }
    }
  };
  // weights of one tile (clamped row ids, zero A past each quarter's end)
  // and the output rows, bias and masks of this lane's four result rows
  struct Tile {
    AF a[OUT_SPLIT][NT];
    int orow[4];
    float b[4], m[NI][4];
  };
  auto load_tile = [&](int row0, Tile& t) {
    // every row id first (one wait), then all the loads that depend on them
    int wrow = min(row0 + rA, nrows - 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) t.orow[i] = min(row0 + 4 * g + i, nrows - 1);
    if (gram) {
      wrow = ldg<int>(cdofs + wrow);
#pragma unroll
      for (int i = 0; i < 4; ++i) t.orow[i] = ldg<int>(cdofs + t.orow[i]);
    }
#pragma unroll
    for (int q = 0; q < OUT_SPLIT; ++q)
#pragma unroll
      for (int s2 = 0; s2 < NT; ++s2) {
        const int kk = q * kq + s2 * KS + (KS / 4) * g;
        const AF v = ldg<AF>(W + (size_t)wrow * K + min(kk, K - KS / 4));
        t.a[q][s2] = kk < (q + 1) * kq ? v : zero_of<AF>();
      }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      t.b[i] = ldg<float>(bias + t.orow[i]);
      t.m[0][i] = use[0] ? ldg<float>(keep0 + t.orow[i]) : 0.f;
      if constexpr (NI > 1) t.m[1][i] = use[1] ? ldg<float>(keep1 + t.orow[i]) : 0.f;
    }
  };
  auto run_tile = [&](int row0, const Tile& t) {
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      if (!use[j]) continue;
      f32x4 acc[OUT_SPLIT][NCB];
#pragma unroll
      for (int q = 0; q < OUT_SPLIT; ++q)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          acc[q][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
          // BF16: K-steps past the quarter's end multiply the zeroed A
          // operand (exact: they add +0), so the unrolled steps carry no
          // branch and their LDS reads are issued ahead of the MFMAs.  FP32
          // skips them (measured: 4% faster at 128 instances than without
          // the branch; BF16 is 1.5% faster without)
#pragma unroll
          for (int s2 = 0; s2 < NT; ++s2) {
            const int k = q * kq + s2 * KS + (KS / 4) * g;
            if (std::is_same<TW, float>::value && s2 * KS >= kq) continue;
            if constexpr (std::is_same<TW, float>::value) {
              const float4 b = *reinterpret_cast<const float4*>(&Fs[j][cb * 16 + rA][min(k, K - 4)]);
              acc[q][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(t.a[q][s2].x, b.x, acc[q][cb], 0, 0, 0);
              acc[q][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(t.a[q][s2].y, b.y, acc[q][cb], 0, 0, 0);
              acc[q][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(t.a[q][s2].z, b.z, acc[q][cb], 0, 0, 0);
              acc[q][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(t.a[q][s2].w, b.w, acc[q][cb], 0, 0, 0);
            } else {
              const float4 b0 = *reinterpret_cast<const float4*>(&Fs[j][cb * 16 + rA][min(k, K - 4)]);
              const float4 b1 = *reinterpret_cast<const float4*>(&Fs[j][cb * 16 + rA][min(k + 4, K - 4)]);
              acc[q][cb] =
                  __builtin_amdgcn_mfma_f32_16x16x32_bf16(t.a[q][s2], to_bf16x8(b0, b1), acc[q][cb], 0, 0, 0);
            }
          }
        }
      // item i of lane l is D[4 (l/16) + i][l % 16]; quarters added in order
      float* rec = j == 0 ? rec0 : rec1;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (row0 + 4 * g + i < nrows) {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) {
            const int c = cb * 16 + rA;
            if (c < Cf) {
              float v = acc[0][cb][i];
#pragma unroll
              for (int q = 1; q < OUT_SPLIT; ++q) v += acc[q][cb][i];
              if (c == 0) v += t.b[i];
              stg<float>(rec + (size_t)t.orow[i] * Cf + c, v * t.m[j][i]);
            }
          }
        }
      }
    }
  };
  const int r0 = blk0 + wave * 16 * OUT_TILES;
  Tile t0, t1;
  load_tile(r0, t0);
  stage_fold();
  __syncthreads();
#pragma unroll
  for (int j = 0; j < OUT_TILES; j += 2) {
    if (j + 1 < OUT_TILES) load_tile(r0 + 16 * (j + 1), t1);
    if (r0 + 16 * j < nrows) run_tile(r0 + 16 * j, t0);
    if (j + 2 < OUT_TILES) load_tile(r0 + 16 * (j + 2), t0);
    if (j + 1 < OUT_TILES && r0 + 16 * (j + 1) < nrows) run_tile(r0 + 16 * (j + 1), t1);
  }
}

// FP64 form of the output layer (plain FMA; correctness configurations)
__global__ __launch_bounds__(256) void k_fwd_out_f64(LayerArgs la, const Inst<double>* __restrict__ tab) {
  const Inst<double>& I = tab[blockIdx.y];
  if (!I.active) return;
  const int K = la.m_inp;
  const int Cf = I.Cf;
  const int nrows = I.gram ? I.n_cdofs : I.N;
  const int pos = blockIdx.x * 16 + (threadIdx.x >> 4);
  const int c0 = threadIdx.x & 15;
  if (pos >= nrows) return;
  const int row = I.gram ? I.cdofs[pos] : pos;
  const double* W = reinterpret_cast<const double*>(la.W) + (size_t)row * K;
  const double* bias = reinterpret_cast<const double*>(la.b);
  for (int c = c0; c < Cf; c += 16) {
    double acc = 0.0;
    const double* f = I.fold + (size_t)c * K;
    for (int k = 0; k < K; ++k) acc = fma(W[k], f[k], acc);
    if (c == 0) acc += bias[row];
    I.rec[(size_t)row * Cf + c] = acc * I.keep[row];
  }
}

// ---------------------------------------------------------------------------
// Filter (I - U U^T) of every output channel and u += U p (n_p > 0 only).
// One block per instance.
// ---------------------------------------------------------------------------
// Filter of every output channel, rec <- (I - U U^T) rec (the mask is
// already applied and U has zero pinned rows), and u = U p + D(q) in the
// value channel when add_up.  Two passes over 256-row blocks: k_filter_part
// writes each block's FP64 partial of Y = U^T rec [n_p][Cf]; k_filter_apply
// adds the partials in block order (every block the same sum) and updates
// its rows.
#define FILT_ROWS 256
template <typename T>
__global__ __launch_bounds__(256) void k_filter_part(const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  const int active = I.active, np = I.n_p, Cf = I.Cf, N = I.N;
  load_now(active, np, Cf, N, I.U, I.rec, I.part_filt);
  if (!active || np == 0) return;
  const int i0 = blockIdx.x * FILT_ROWS;
  if (i0 >= N) return;
  const int nr = min(FILT_ROWS, N - i0);
  // rows staged 64 at a time; thread t accumulates entries t + 256 j of
  // [n_p][Cf] (at most 8) over the rows in order
  constexpr int CH = 64, EPT = (NMR_MAX_R * 64 + 255) / 256;
  __shared__ double sU[CH][NMR_MAX_R + 1];
  __shared__ double sR[CH][65];
  double acc[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) acc[j] = 0.0;
  for (int r0 = 0; r0 < nr; r0 += CH) {
    const int nc = min(CH, nr - r0);
    for (int e = threadIdx.x; e < nc * np; e += 256) {
      const int i = e / np, k = e - i * np;
      sU[i][k] = (double)ldg<T>(I.U + (size_t)(i0 + r0 + i) * np + k);
    }
    for (int e = threadIdx.x; e < nc * Cf; e += 256) {
      const int i = e / Cf, c = e - i * Cf;
      sR[i][c] = (double)ldg<T>(I.rec + (size_t)(i0 + r0 + i) * Cf + c);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = threadIdx.x + 256 * j;
      if (e < np * Cf) {
        const int k = e / Cf, c = e - k * Cf;
        for (int i = 0; i < nc; ++i) acc[j] = fma(sU[i][k], sR[i][c], acc[j]);
      }
    }
    __syncthreads();
  }
  double* out = I.part_filt + (size_t)blockIdx.x * np * Cf;
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = threadIdx.x + 256 * j;
    if (e < np * Cf) stg<double>(out + e, acc[j]);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_filter_apply(const Inst<T>* __restrict__ tab, int add_up) {
  const Inst<T>& I = tab[blockIdx.y];
  const int active = I.active, np = I.n_p, Cf = I.Cf, N = I.N;
  load_now(active, np, Cf, N, I.U, I.rec, I.part_filt, I.r);
  if (!active || np == 0) return;
  const int i0 = blockIdx.x * FILT_ROWS;
  if (i0 >= N) return;
  const int nblk = (N + FILT_ROWS - 1) / FILT_ROWS;
  __shared__ double Y[NMR_MAX_R][65];
  __shared__ double pv[NMR_MAX_R];
  for (int e = threadIdx.x; e < np * Cf; e += 256) {
    const int k = e / Cf, c = e - k * Cf;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += ldg<double>(I.part_filt + (size_t)b * np * Cf + e);
    Y[k][c] = acc;
  }
  if (threadIdx.x < np) pv[threadIdx.x] = ldg<double>(I.r + threadIdx.x);
  __syncthreads();
  const int nr = min(FILT_ROWS, N - i0);
  for (int e = threadIdx.x; e < nr * Cf; e += 256) {
    const int i = i0 + e / Cf, c = e % Cf;
    T* rp = I.rec + (size_t)i * Cf + c;
    double v = (double)ldg<T>(rp);
    for (int k = 0; k < np; ++k) v -= (double)ldg<T>(I.U + (size_t)i * np + k) * Y[k][c];
    if (c == 0 && add_up)
      for (int k = 0; k < np; ++k) v += (double)ldg<T>(I.U + (size_t)i * np + k) * pv[k];
    stg<T>(rp, (T)v);
  }
}

// ---------------------------------------------------------------------------
// Backward through the output layer: partial sums of W_L^T s over 128-row
// chunks, s_i = seed_i - sum_k U_ik (U^T P a)_k (the filter's transpose).
// 64 column groups of 4 x 4 row slices per block; slices added in order.
// ---------------------------------------------------------------------------
#define BWD_ROWS 128
__device__ inline void load4(const float* p, double (&w)[4]) {
  const float4 v = ldg<float4>(p);
  w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
}
__device__ inline void load4(const double* p, double (&w)[4]) {
  const double2 v01 = ldg<double2>(p), v23 = ldg<double2>(p + 2);
  const double4 v = make_double4(v01.x, v01.y, v23.x, v23.y);
  w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
}
__device__ inline void load4(const __bf16* p, double (&w)[4]) {
  const bf16x4 v = ldg<bf16x4>(p);
  w[0] = (float)v[0]; w[1] = (float)v[1]; w[2] = (float)v[2]; w[3] = (float)v[3];
}

template <typename T, typename TW>
__device__ __forceinline__ void bwd_out_block(const LayerArgs& la, const Inst<T>* __restrict__ tab, int bx, int by) {
  const Inst<T>& I = tab[by];
  load_now(I.active, I.gram, I.n_sblk, I.n_bblk, I.n_cdofs, I.N, I.n_p, I.R, I.n_q, I.sum_mass, I.cdofs, I.keep,
           I.seed, I.U, I.part_bwd, I.csr_ptr, I.csr_ent, I.fe, la.m_inp, la.W);
  if (!I.active) return;
  // direct path: all N rows with the seed P a (and the filter transpose);
  // Gram path: only the cubature DOFs with dt^2 P f_int (the rest of W_L^T P a
  // is Gam y + gam, added by the Gram kernel as one more partial)
  if (bx >= (I.gram ? I.n_sblk : I.n_bblk)) return;
  const int K = la.m_inp;
  const int nrows = I.gram ? I.n_cdofs : I.N;
  const int i0 = bx * BWD_ROWS;
  const int i1 = min(i0 + BWD_ROWS, nrows);
  __shared__ double s[BWD_ROWS];
  __shared__ int srow[BWD_ROWS];
  __shared__ double red[4][256];
  const int np = I.n_p;
  const double* uta = I.sum_mass + I.R * I.R + I.R * I.n_q + I.R;
  for (int i = i0 + threadIdx.x; i < i1; i += 256) {
    double v;
    int row = i;
    if (I.gram) {
      row = ldg<int>(I.cdofs + i);
      v = I.dt * I.dt * (double)ldg<T>(I.keep + row) * fint_at(I, row);
    } else {
      v = (double)ldg<T>(I.seed + i);
      for (int k = 0; k < np; ++k) v -= (double)ldg<T>(I.U + (size_t)i * np + k) * ldg<double>(uta + k);
    }
    s[i - i0] = v;
    srow[i - i0] = row;
  }
  __syncthreads();
  const TW* W = reinterpret_cast<const TW*>(la.W);
  const int cg = threadIdx.x & 63, sl = threadIdx.x >> 6;
  for (int c0 = 0; c0 < K; c0 += 256) {
    const int col = c0 + 4 * cg;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (col < K) {
#pragma unroll 8
      for (int i = i0 + sl; i < i1; i += 4) {
        double w[4];
        load4(W + (size_t)srow[i - i0] * K + col, w);
        const double si = s[i - i0];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = fma(w[t], si, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) red[sl][4 * cg + t] = acc[t];
    __syncthreads();
    const int c = c0 + threadIdx.x;
    if (c < K)
      stg<double>(I.part_bwd + (size_t)bx * K + c,
                  ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x]);
    __syncthreads();
  }
}

template <typename T, typename TW>
__global__ __launch_bounds__(256) void k_bwd_out(LayerArgs la, const Inst<T>* __restrict__ tab) {
  bwd_out_block<T, TW>(la, tab, blockIdx.x, blockIdx.y);
}

// The Gram path's output-layer backpropagation for instances that decode the
// same rows (`rows`, shared by every member of the launch): a block takes
// 128 rows and BWD_NJ instances, so every weight row it loads serves all of
// them.  Each instance's partial is the same sum in the same order as in
// bwd_out_block (slice sl adds rows i0 + sl, i0 + sl + 4, ...; slices
// combined in order), so the results are the same bits.  Slots not in use
// contribute nothing and their pointers are never read.
#define BWD_NJ 8
template <typename TW>
__global__ __launch_bounds__(256) void k_bwd_out_batch(LayerArgs la, const Inst<float>* __restrict__ tab, int nb,
                                                       const int* __restrict__ rows, int nrows) {
  const int bx = blockIdx.x, j0 = blockIdx.y * BWD_NJ, tid = threadIdx.x;
  const int K = la.m_inp;
  const int i0 = bx * BWD_ROWS;
  if (i0 >= nrows) return;
  const int i1 = min(i0 + BWD_ROWS, nrows), ni = i1 - i0;
  __shared__ double s[BWD_NJ][BWD_ROWS];
  __shared__ int srow[BWD_ROWS];
  __shared__ int sact[BWD_NJ];
  __shared__ double red[4][256];
  if (tid < BWD_NJ) {
    const int j = j0 + tid;
    sact[tid] = (j < nb && tab[j].active && tab[j].gram) ? 1 : 0;
  }
  for (int i = tid; i < ni; i += 256) srow[i] = ldg<int>(rows + i0 + i);
  __syncthreads();
  for (int e = tid; e < BWD_NJ * ni; e += 256) {
    const int jj = e / ni, ii = e - jj * ni;
    double v = 0.0;
    if (sact[jj]) {
      const Inst<float>& I = tab[j0 + jj];
      const int row = srow[ii];
      v = I.dt * I.dt * (double)ldg<float>(I.keep + row) * fint_at(I, row);
    }
    s[jj][ii] = v;
  }
  __syncthreads();
  const TW* W = reinterpret_cast<const TW*>(la.W);
  const int cg = tid & 63, sl = tid >> 6, col = 4 * cg;
  double acc[BWD_NJ][4];
#pragma unroll
  for (int jj = 0; jj < BWD_NJ; ++jj)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[jj][t] = 0.0;
  if (col < K) {
#pragma unroll 4
    for (int i = i0 + sl; i < i1; i += 4) {
      double w[4];
      load4(W + (size_t)srow[i - i0] * K + col, w);
#pragma unroll
      for (int jj = 0; jj < BWD_NJ; ++jj) {
        const double si = s[jj][i - i0];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[jj][t] = fma(w[t], si, acc[jj][t]);
      }
    }
  }
#pragma unroll
  for (int jj = 0; jj < BWD_NJ; ++jj) {
#pragma unroll
    for (int t = 0; t < 4; ++t) red[sl][4 * cg + t] = acc[jj][t];
    __syncthreads();
    if (sact[jj] && tid < K)
      stg<double>(tab[j0 + jj].part_bwd + (size_t)bx * K + tid, ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid]);
    __syncthreads();
  }
}

// The partial sums and the output-layer backpropagation in one launch (Gram
// path: the seed dt^2 P f_int needs the element forces, not the sums):
// blocks below n_sum run the sums, the rest the output-layer rows.
template <typename T, typename TW>
__global__ __launch_bounds__(256) void k_sums_bwd_out(LayerArgs la, const Inst<T>* __restrict__ tab, int cub_m,
                                                      int n_sum) {
  if ((int)blockIdx.x < n_sum) sums_block<T>(tab, blockIdx.x, blockIdx.y, cub_m);
  else bwd_out_block<T, TW>(la, tab, blockIdx.x - n_sum, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Sum the output-layer partials (fixed order) and apply sigma' of the last
// hidden layer: xb0 = s1 zb0, xb1_j = s2 x1_j zb0 (the seed is real).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_reduce(LayerArgs la, const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  load_now(I.active, I.gram, I.fd, I.n_sblk, I.n_bblk, I.part_bwd, I.pre[la.l - 1], I.zb0, I.n_q, la.m_inp,
           la.m_in, la.act);
  if (!I.active) return;
  const int l = la.l;  // output layer; its input is hidden layer l-1
  const int K = la.m_inp;
  const int kk = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const int k = blockIdx.x * 16 + kk;
  const int nch = I.fd ? 1 + 2 * I.n_q : 1 + I.n_q;  // real backpropagation columns / value + e_j tangents
  const T* pre = I.pre[l - 1];
  __shared__ double part[16][17];
  // every load leaves before the first wait: the partials of slice sl and
  // the pre-activations of this thread's channels (sl, sl + 16) at column k
  const int kc = min(k, K - 1);
  const T x0 = ldg<T>(pre + kc);
  const T xa = ldg<T>(pre + (size_t)min(sl, nch - 1) * K + kc);
  const T xb2 = ldg<T>(pre + (size_t)min(sl + 16, nch - 1) * K + kc);
  double acc = 0.0;
  if (k < K) {
    const double* src = I.part_bwd + k;
    const int nb = I.gram ? I.n_sblk + kGramKParts : I.n_bblk;  // Gram: + the Gam y (+ gam) partials
#pragma unroll 4
    for (int b = sl; b < nb; b += 16) acc += ldg<double>(src + (size_t)b * K);
  }
  part[sl][kk] = acc;
  __syncthreads();
  if (k >= K) return;
  double zb0 = part[0][kk];
  for (int q = 1; q < 16; ++q) zb0 += part[q][kk];
  T* xb = I.zb0;
  const bool in = k < la.m_in;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = sl + 16 * h;
    if (c >= nch) break;
    const T xc = h == 0 ? xa : xb2;
    T v;
    if (I.fd) {
      // real backpropagation of every kept stencil column (base, q +- h e_j)
      T d1, d2;
      act_d12(la.act, xc, d1, d2);
      v = (T)(d1 * zb0);
    } else {
      T d1, d2;
      act_d12(la.act, x0, d1, d2);
      v = c == 0 ? (T)(d1 * zb0) : (T)(d2 * xc * zb0);
    }
    if (la.bf16 && !I.fd) stg<__bf16>(reinterpret_cast<__bf16*>(xb) + (size_t)c * K + k, (__bf16)(float)(in ? v : T(0)));
    else stg<T>(xb + (size_t)c * K + k, in ? v : T(0));
  }
}

// ---------------------------------------------------------------------------
// Backward through hidden layer l: zb_prev = W_l^T xb_l (split-K GEMM with the
// transposed weights stored row-major), then either sigma' of layer l-1 or,
// at the input, J^T a and a . H.
// ---------------------------------------------------------------------------
template <typename T, typename TW, int NCB, int IB, bool FD, int MR>
__global__ __launch_bounds__(MR > 1 ? 64 * IB * (tall_ks<TW, NCB, MR>::v) : 512) void k_bwd_hidden(LayerArgs la,
                                                                                       const Inst<T>* __restrict__ tab,
                                                                                       int nb) {
  static_assert(MR == 1 || (!FD && std::is_same<T, float>::value), "tall tiles: complex-step FP32 jets only");
  constexpr int ROWS = 16 * MR;  // rows (layer inputs) of a block
  constexpr int NW = MR > 1 ? IB * tall_ks<TW, NCB, MR>::v : splitk_waves<T, NCB>::v;
  constexpr int KSPL = NW / IB;
  constexpr int NG = KSPL * 64;  // threads of one instance slot
  const int l = la.l;
  const int step = la.L - 2 - l;  // 0 for the last hidden layer
  const int tid = threadIdx.x, wave = tid >> 6;
  const int slot = wave / KSPL, tg = tid - slot * NG;
  int bx = blockIdx.x, by = blockIdx.y;  // whole instance groups per XCD
  if (gridDim.y > 1) xcd_block(bx, by);
  const int inst = by * IB + slot;
  const Inst<T>& I = tab[min(inst, nb - 1)];
  // the table entry's fields are read before any test so that their scalar
  // loads leave together
  constexpr bool fd = FD;  // central differences instead of complex-step jets
  const int active = I.active, nq = I.n_q;
  const T* xb = (step & 1) ? I.zb1 : I.zb0;
  T* const xb_out = (step & 1) ? I.zb0 : I.zb1;
  const T* pre = (l > 0) ? I.pre[l - 1] : nullptr;
  double* const JTa = I.JTa;
  double* const Bq = I.Bq;
  const double fdh64 = I.fd_h;
  const int K = la.m_outp;  // reduction over the outputs of layer l
  const int m_in = la.m_in, m_inp = la.m_inp;
  load_now(active, nq, xb, xb_out, pre, JTa, Bq, fdh64, K, m_in, m_inp, la.WT, la.act);
  // channels: value and the e_j tangents (complex steps), or the base and
  // q +- h e_j stencil columns (central differences)
  const int nch = fd ? 1 + 2 * nq : 1 + nq;
  const bool use = inst < nb && active;
  const int row0 = bx * ROWS;
  if (row0 >= m_inp || (IB == 1 && !use)) return;  // uniform over the block
  const TW* WT = reinterpret_cast<const TW*>(la.WT) + (size_t)row0 * K;
  using STG = tall_stage<TW, NCB, MR, IB, tall_ks<TW, NCB, MR>::v>;
  constexpr int SB = (int)sizeof(T) * IB * NCB * 16 * (ROWS + 1), GB = STG::on ? STG::BYTES : 0;
  __shared__ __align__(16) unsigned char lds_s[SB > GB ? SB : GB];  // S, or the GEMM's staging before it
  T(*S)[NCB * 16][ROWS + 1] = reinterpret_cast<T(*)[NCB * 16][ROWS + 1]>(lds_s);
  __shared__ T red[MR == 1 ? NW : 1][NCB * 16][16];
  typedef typename vec4<T>::type V4;
  // a BF16 decoder's adjoints are stored as BF16 (complex-step BP only)
  constexpr bool BFX = std::is_same<TW, __bf16>::value && !FD;
  auto bload = [&](int c, int k) {
    if constexpr (BFX) return ldg<bf16x8>(reinterpret_cast<const __bf16*>(xb) + (size_t)c * K + k);
    else return ldg<V4>(xb + (size_t)c * K + k);
  };
  // pre-activations of layer l-1 used by the epilogue, loaded before the GEMM
  // (an item: VG consecutive rows of a channel; tall tiles store 16 bytes)
  constexpr int VG = MR == 1 ? 1 : BFX ? 8 : 4, RG = ROWS / VG;
  constexpr int PP = (RG * 32 + NG - 1) / NG;  // items per thread: RG row groups x (nch <= 32) channels
  T px0[PP][VG], px1[PP][VG];
#pragma unroll
  for (int t = 0; t < PP; ++t) {
    const int p = tg + t * NG;
#pragma unroll
    for (int i = 0; i < VG; ++i) px0[t][i] = px1[t][i] = T(0);
    if (use && l > 0 && p < RG * nch) {
      const int c = p / RG, r = VG * (p - c * RG);
      if constexpr (VG == 1) {
        px0[t][0] = ldg<T>(pre + row0 + r);
        if (c > 0) px1[t][0] = ldg<T>(pre + (size_t)c * m_inp + row0 + r);
      } else
#pragma unroll
      for (int h = 0; h < VG; h += 4) {
        const V4 a = ldg<V4>(pre + row0 + r + h);
        px0[t][h] = a.x; px0[t][h + 1] = a.y; px0[t][h + 2] = a.z; px0[t][h + 3] = a.w;
        if (c > 0) {
          const V4 b = ldg<V4>(pre + (size_t)c * m_inp + row0 + r + h);
          px1[t][h] = b.x; px1[t][h + 1] = b.y; px1[t][h + 2] = b.z; px1[t][h + 3] = b.w;
        }
      }
    }
  }
  if constexpr (MR == 1) gemm_splitk<T, TW, NCB, NW, IB>(WT, K, K, use, bload, S, red);
  else if constexpr (STG::on)
    gemm_tall_lds<TW, NCB, MR, IB, tall_ks<TW, NCB, MR>::v>(WT, K, K, use, reinterpret_cast<const TW*>(xb), K, S, lds_s);
  else gemm_tall<TW, NCB, MR, tall_ks<TW, NCB, MR>::v>(WT, K, K, use, bload, S);
  if (!use) return;
  T(*Ss)[ROWS + 1] = S[slot];
  if (l > 0) {
#pragma unroll
    for (int t = 0; t < PP; ++t) {
      const int p = tg + t * NG;
      if (p < RG * nch) {
        const int c = p / RG, r = VG * (p - c * RG);
        T v[VG];
#pragma unroll
        for (int i = 0; i < VG; ++i) {
          T d1, d2;
          if constexpr (FD) {  // each column through sigma' of its own pre-activation
            act_d12(la.act, c == 0 ? px0[t][i] : px1[t][i], d1, d2);
            v[i] = d1 * Ss[c][r + i];
          } else {
            act_d12(la.act, px0[t][i], d1, d2);
            if (c == 0) v[i] = d1 * Ss[0][r + i];
            else v[i] = d1 * Ss[c][r + i] + d2 * px1[t][i] * Ss[0][r + i];
          }
          v[i] = (row0 + r + i < m_in) ? v[i] : T(0);
        }
        if constexpr (VG == 1) {
          if constexpr (BFX) stg<__bf16>(reinterpret_cast<__bf16*>(xb_out) + (size_t)c * m_inp + row0 + r, (__bf16)v[0]);
          else stg<T>(xb_out + (size_t)c * m_inp + row0 + r, v[0]);
        } else if constexpr (BFX) {
          bf16x8 o;
#pragma unroll
          for (int i = 0; i < 8; ++i) o[i] = (__bf16)v[i];
          stg<bf16x8>(reinterpret_cast<__bf16*>(xb_out) + (size_t)c * m_inp + row0 + r, o);
        } else {
          stg<V4>(xb_out + (size_t)c * m_inp + row0 + r, V4{v[0], v[1], v[2], v[3]});
        }
      }
    }
  } else {
    for (int p = tg; p < ROWS * (1 + nq); p += NG) {
      const int r = p & (ROWS - 1), c = p / ROWS;
      const int row = row0 + r;
      if (row < nq) {
        if (c == 0) stg<double>(JTa + row, (double)Ss[0][r]);
        else if constexpr (FD)  // (grad at q + h e_j - grad at q - h e_j) / 2h
          stg<double>(Bq + (size_t)row * nq + (c - 1),
                      (double)((Ss[2 * c - 1][r] - Ss[2 * c][r]) / (T(2) * (T)fdh64)));
        else stg<double>(Bq + (size_t)row * nq + (c - 1), (double)Ss[c][r]);
      }
    }
  }
}

// rec -> separate u, J, dJ, Hdd arrays (decoder_jacobian_hessian outputs)
template <typename T>
__global__ void k_unpack(const Inst<T>* __restrict__ tab, T* u, T* J, T* dJ, T* Hdd) {
  const Inst<T>& I = tab[0];
  const int nq = I.n_q, Cf = I.Cf;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= I.N) return;
  const T* rr = I.rec + (size_t)i * Cf;
  if (u) u[i] = rr[0];
  for (int j = 0; j < nq; ++j) {
    if (J) J[(size_t)i * nq + j] = rr[1 + j];
    if (dJ) dJ[(size_t)i * nq + j] = rr[1 + nq + j];
  }
  if (Hdd) Hdd[i] = rr[1 + 2 * nq];
}

// ---------------------------------------------------------------------------
// Frame output: the full-space displacement u of the state the forward pass
// was run at (dq = 0 there, so the value channel is u itself).  Gram path
// (n_p = 0): u_i = keep_i (W_L[i,:] . fold_value + b_i) for every DOF, a
// memory-bound GEMV; 16 lanes per row, each reading 4 consecutive K entries
// per step (one 64-entry K slice per step across the 16 lanes), then a
// butterfly sum within the 16 lanes.  Direct path: the records already hold
// u = U p + D(q) in their value channel.
// ---------------------------------------------------------------------------
template <typename T, typename TW>
__global__ __launch_bounds__(256) void k_frame(LayerArgs la, const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  const int active = I.active, gram = I.gram, N = I.N, Cf = I.Cf;
  const T* fold = I.fold;
  const T* rec = I.rec;
  const T* keep = I.keep;
  T* frame = I.frame;
  const int K = la.m_inp;
  load_now(active, gram, N, Cf, fold, rec, keep, frame, K, la.W, la.b);
  if (!active) return;
  if (!gram) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < N) stg<T>(frame + i, ldg<T>(rec + (size_t)i * Cf));
    return;
  }
  const int row = blockIdx.x * 16 + (threadIdx.x >> 4), j = threadIdx.x & 15;
  if (blockIdx.x * 16 >= N) return;  // uniform over the block
  const int rr = min(row, N - 1);
  const TW* w = reinterpret_cast<const TW*>(la.W) + (size_t)rr * K;
  typedef typename std::conditional<std::is_same<T, double>::value, double, float>::type Acc;
  Acc acc = Acc(0);
  for (int k = 4 * j; k < K; k += 64) {
    typedef typename vec4<T>::type V4;
    const V4 x = ldg<V4>(fold + k);
    Acc w0, w1, w2, w3;
    if constexpr (std::is_same<TW, __bf16>::value) {
      const bf16x4 v = ldg<bf16x4>(w + k);
      w0 = (Acc)(float)v[0]; w1 = (Acc)(float)v[1]; w2 = (Acc)(float)v[2]; w3 = (Acc)(float)v[3];
    } else {
      const V4 v = ldg<V4>(w + k);
      w0 = v.x; w1 = v.y; w2 = v.z; w3 = v.w;
    }
    acc += w0 * (Acc)x.x + w1 * (Acc)x.y + w2 * (Acc)x.z + w3 * (Acc)x.w;
  }
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 16);
  if (j == 0 && row < N) {
    const T b = ldg<T>(reinterpret_cast<const T*>(la.b) + row);
    stg<T>(frame + row, (T)((acc + (Acc)b) * (Acc)ldg<T>(keep + row)));
  }
}

// Frames of many instances sharing a decoder (Gram path): one GEMM with the
// instances as columns, U = W_L [F_0 ... F_nb] for the value channels F_j of
// the folded activations, so every weight row is read once for all of them.
// A block takes 256 rows (four waves of four 16-row tiles) and 32 instance
// columns, whose value channels it stages in LDS (zeros for a slot not in
// use, whose pointers are never read).  u_j[i] = keep_j[i] (acc + b_i) for
// rows i < N_j.
#define FRAME_COLS 32
template <typename TW>
__global__ __launch_bounds__(256) void k_frame_batch(LayerArgs la, const Inst<float>* __restrict__ tab, int nb) {
  constexpr int NCB = FRAME_COLS / 16;
  const int K = la.m_inp;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rA = lane & 15, g = lane >> 4;
  const int c0 = blockIdx.y * FRAME_COLS;
  __shared__ __align__(16) float Fs[FRAME_COLS][OUT_KMAX + 4];
  __shared__ int s_act[FRAME_COLS], s_n[FRAME_COLS];
  if (threadIdx.x < FRAME_COLS) {
    const int j = c0 + threadIdx.x;
    const int act = j < nb ? tab[j].active : 0;
    s_act[threadIdx.x] = act && tab[j].gram;
    s_n[threadIdx.x] = act ? tab[j].N : 0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < FRAME_COLS * (K / 4); e += 256) {
    const int c = e / (K / 4), k = 4 * (e - c * (K / 4));
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (s_act[c]) v = ldg<float4>(tab[c0 + c].fold + k);
    *reinterpret_cast<float4*>(&Fs[c][k]) = v;
  }
  __syncthreads();
  const TW* W = reinterpret_cast<const TW*>(la.W);
  const float* bias = reinterpret_cast<const float*>(la.b);
  const int m_out = la.m_out;
  for (int t = 0; t < 4; ++t) {
    const int row0 = blockIdx.x * 256 + wave * 64 + t * 16;
    if (row0 >= m_out) break;  // uniform over the wave
    const int wrow = min(row0 + rA, m_out - 1);
    f32x4 acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (std::is_same<TW, float>::value) {
      for (int k = 0; k < K; k += 16) {
        const float4 a = ldg<float4>(W + (size_t)wrow * K + k + 4 * g);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const float4 b = *reinterpret_cast<const float4*>(&Fs[cb * 16 + rA][k + 4 * g]);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[cb], 0, 0, 0);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[cb], 0, 0, 0);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc[cb], 0, 0, 0);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc[cb], 0, 0, 0);
        }
      }
    } else {
      for (int k = 0; k < K; k += 32) {
        const bf16x8 a = ldg<bf16x8>(W + (size_t)wrow * K + k + 8 * g);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const float4 b0 = *reinterpret_cast<const float4*>(&Fs[cb * 16 + rA][k + 8 * g]);
          const float4 b1 = *reinterpret_cast<const float4*>(&Fs[cb * 16 + rA][k + 8 * g + 4]);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, to_bf16x8(b0, b1), acc[cb], 0, 0, 0);
        }
      }
    }
    // item i of lane l is D[4 (l/16) + i][l % 16]: row row0 + 4 g + i of
    // instance c0 + cb * 16 + rA
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int c = cb * 16 + rA;
      if (!s_act[c]) continue;
      const Inst<float>& I = tab[c0 + c];
      float* frame = I.frame;
      const float* keep = I.keep;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = row0 + 4 * g + i;
        if (row < s_n[c]) stg<float>(frame + row, (acc[cb][i] + ldg<float>(bias + row)) * ldg<float>(keep + row));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define NCB_SWITCH(ncb, CALL) \
  switch (ncb) {              \
    case 1: CALL(1); break;   \
    case 2: CALL(2); break;   \
    case 3: CALL(3); break;   \
    case 4: CALL(4); break;   \
    case 5: CALL(5); break;   \
    case 6: CALL(6); break;   \
    case 7: CALL(7); break;   \
    case 8: CALL(8); break;   \
    default: break;           \
  }

// ---------------------------------------------------------------------------
// tile configurations of the hidden-layer launches
// ---------------------------------------------------------------------------
static int hidden_rows(const DecoderDev& d, int l, bool fwd) { return fwd ? d.wp[l + 1] : d.wp[l]; }

// columns a tall tile holds in registers: MR x NCB accumulators and two
// K-batches of MR + NCB operand fragments per wave
static int tall_max_cols(int mr, bool fwd) { return fwd ? (mr == 2 ? 128 : 64) : 32; }

// perturbations per jet group, and the groups of a decoder's input width
static constexpr int kJetGroup = 3;
// tall tiles from this many (row tile, instance) waves
static constexpr int kTallWaves = 768;
static int jet_groups(const DecoderDev& d) { return (d.w[0] + kJetGroup - 1) / kJetGroup; }

// Layers with tall tiles (at most 64 jet columns forward, 32 adjoint columns
// backward) take them once there are 768 (row tile, instance) waves of 16 mr
// rows, the largest mr first; otherwise instances are stacked as above.
// Forward layers whose (row tile, instance) blocks leave most CUs idle split
// the jet columns into groups instead.  Both crossovers are the ones the
// autotuner finds on the 10k-vertex decoder from 8 to 128 instances.
TileCfg tile_rule(const DecoderDev& d, int l, int nb, int cols, bool fd, bool f64, bool fwd) {
  if (fd || f64) return TileCfg{1, 1};
  const int rows = hidden_rows(d, l, fwd);
  if (nb >= 4)
    for (int mr = 4; mr >= 2; mr /= 2)
      if (cols <= tall_max_cols(mr, fwd) && rows % (16 * mr) == 0 && (rows / (16 * mr)) * nb >= kTallWaves)
        return TileCfg{4, mr};
  const int ib = stack_instances(rows / 16, nb, false);
  if (ib == 1 && fwd && cols > 16 && (rows / 16) * nb < kJetGroupBlocks) return TileCfg{1, 1, 1};
  return TileCfg{ib, 1};
}

bool tile_eligible(const DecoderDev& d, int l, int nb, int cols, bool fd, bool f64, bool fwd, TileCfg c) {
  if (c.jg) return c.ib == 1 && c.mr == 1 && fwd && !fd && !f64 && cols > 16 && nb * jet_groups(d) <= 65535;
  if (c.ib == 1 && c.mr == 1) return true;
  if (fd || f64 || nb < c.ib) return false;
  if (c.mr == 1) return c.ib == 2 || c.ib == 4;
  return c.ib == 4 && (c.mr == 2 || c.mr == 4) && cols <= tall_max_cols(c.mr, fwd) &&
         hidden_rows(d, l, fwd) % (16 * c.mr) == 0;
}

int tile_candidates(const DecoderDev& d, int l, int nb, int cols, bool fd, bool f64, bool fwd, TileCfg* out) {
  static const TileCfg all[] = {{1, 1}, {1, 1, 1}, {2, 1}, {4, 1}, {4, 2}, {4, 4}};
  int n = 0;
  for (const TileCfg& c : all)
    if (tile_eligible(d, l, nb, cols, fd, f64, fwd, c)) out[n++] = c;
  return n;
}

template <typename T, typename TW, int NCB>
static void fwd_hidden_ib(const DecoderDev& d, int l, const Inst<T>* tab, int nb, bool fd, TileCfg cfg,
                          hipStream_t s) {
  const int rows = d.wp[l + 1], tiles = rows / 16;
  const int threads = 64 * splitk_waves<T, NCB>::v;
  const LayerArgs la = layer_args(d, l);
  if (fd) {  // the central-difference form: one instance per block
    k_fwd_hidden<T, TW, NCB, 1, true, 1><<<dim3(tiles, nb), threads, 0, s>>>(la, tab, nb);
    return;
  }
  if constexpr (std::is_same<T, float>::value) {
    if (cfg.jg) {
      k_fwd_hidden<T, TW, 1, 1, false, 1, kJetGroup><<<dim3(tiles, nb * jet_groups(d)), 512, 0, s>>>(la, tab, nb);
      return;
    }
  }
  if constexpr (std::is_same<T, float>::value && NCB <= 4) {
    if (cfg.mr == 4) {
      k_fwd_hidden<T, TW, NCB, 4, false, 4><<<dim3(rows / 64, (nb + 3) / 4), 256 * tall_ks<TW, NCB, 4>::v, 0, s>>>(la, tab, nb);
      return;
    }
  }
  if constexpr (std::is_same<T, float>::value && NCB <= 8) {
    if (cfg.mr == 2) {
      k_fwd_hidden<T, TW, NCB, 4, false, 2><<<dim3(rows / 32, (nb + 3) / 4), 256 * tall_ks<TW, NCB, 2>::v, 0, s>>>(la, tab, nb);
      return;
    }
  }
  if (cfg.ib == 4) k_fwd_hidden<T, TW, NCB, 4, false, 1><<<dim3(tiles, (nb + 3) / 4), threads, 0, s>>>(la, tab, nb);
  else if (cfg.ib == 2)
    k_fwd_hidden<T, TW, NCB, 2, false, 1><<<dim3(tiles, (nb + 1) / 2), threads, 0, s>>>(la, tab, nb);
  else k_fwd_hidden<T, TW, NCB, 1, false, 1><<<dim3(tiles, nb), threads, 0, s>>>(la, tab, nb);
}

template <typename T, typename TW>
static void fwd_hidden_dispatch(const DecoderDev& d, int l, const Inst<T>* tab, int nb, int cp, bool fd,
                                TileCfg cfg, hipStream_t s) {
#define FWD_H(n) fwd_hidden_ib<T, TW, n>(d, l, tab, nb, fd, cfg, s)
  NCB_SWITCH(cp / 16, FWD_H)
#undef FWD_H
}

// cfg.ib == 0, or a configuration the layer cannot run: the rule
static TileCfg resolve(const DecoderDev& d, int l, int nb, int cols, bool fd, bool f64, bool fwd, TileCfg cfg) {
  if (cfg.ib == 0 || !tile_eligible(d, l, nb, cols, fd, f64, fwd, cfg)) return tile_rule(d, l, nb, cols, fd, f64, fwd);
  return cfg;
}

template <>
void launch_fwd_hidden<float>(const DecoderDev& d, int l, const Inst<float>* tab, int nb, int cp, bool fd,
                              TileCfg cfg, hipStream_t s) {
  cfg = resolve(d, l, nb, cp, fd, false, true, cfg);
  if (d.prec == PREC_BF16) fwd_hidden_dispatch<float, __bf16>(d, l, tab, nb, cp, fd, cfg, s);
  else fwd_hidden_dispatch<float, float>(d, l, tab, nb, cp, fd, cfg, s);
}
template <>
void launch_fwd_hidden<double>(const DecoderDev& d, int l, const Inst<double>* tab, int nb, int cp, bool fd,
                               TileCfg, hipStream_t s) {
  // FP64 decoders take n_q <= 15, i.e. at most 4 column blocks; one instance per block
  dim3 grid(d.wp[l + 1] / 16, nb);
#define FWD_H64(n)                                                                                                \
  do {                                                                                                           \
    if (fd)                                                                                                      \
      k_fwd_hidden<double, double, n, 1, true, 1><<<grid, 64 * splitk_waves<double, n>::v, 0, s>>>(              \
          layer_args(d, l), tab, nb);                                                                            \
    else                                                                                                         \
      k_fwd_hidden<double, double, n, 1, false, 1><<<grid, 64 * splitk_waves<double, n>::v, 0, s>>>(             \
          layer_args(d, l), tab, nb);                                                                            \
  } while (0)
  switch (cp / 16) {
    case 1: FWD_H64(1); break;
    case 2: FWD_H64(2); break;
    case 3: FWD_H64(3); break;
    case 4: FWD_H64(4); break;
    default: break;
  }
#undef FWD_H64
}

// the wide form once the instances fill the chip with OUT_TILES-fold fewer
// blocks; two instances per block when they decode the same rows and there
// are enough of them
static bool fwd_out_wide(int max_n, int nb) { return nb >= 8 && ((max_n + 127) / 128) * nb >= 1024; }

template <typename TW>
static void fwd_out_dispatch(const DecoderDev& d, const Inst<float>* tab, int nb, int max_n, int cf, bool same_rows,
                             const int* rows, hipStream_t s) {
  const bool wide = fwd_out_wide(max_n, nb);
  const bool pair = wide && (same_rows || rows) && ((max_n + 127) / 128) * ((nb + 1) / 2) >= 1024;
  const int n_rg = (max_n + 16 * OUT_SPLIT * OUT_TILES - 1) / (16 * OUT_SPLIT * OUT_TILES);
  const dim3 grid((max_n + 15) / 16, nb), gridw(n_rg, nb), gridp(n_rg, (nb + 1) / 2);
  const LayerArgs la = layer_args(d, d.L - 1);
#define FWD_O(n)                                                                       \
  do {                                                                                 \
    if (pair) k_fwd_out_wide<TW, n, 2><<<gridp, OUT_SPLIT * 64, 0, s>>>(la, tab, nb, rows);  \
    else if (wide) k_fwd_out_wide<TW, n, 1><<<gridw, OUT_SPLIT * 64, 0, s>>>(la, tab, nb, rows); \
    else k_fwd_out<TW, n><<<grid, OUT_SPLIT * 64, 0, s>>>(la, tab);                     \
  } while (0)
  switch (cf / 16) {
    case 1: FWD_O(1); break;
    case 2: FWD_O(2); break;
    case 3: FWD_O(3); break;
    case 4: FWD_O(4); break;
    default: break;
  }
#undef FWD_O
}

template <>
void launch_fwd_out<float>(const DecoderDev& d, const Inst<float>* tab, int nb, int max_n, int cf, bool same_rows,
                           const int* rows, hipStream_t s) {
  if (d.prec == PREC_BF16) fwd_out_dispatch<__bf16>(d, tab, nb, max_n, cf, same_rows, rows, s);
  else fwd_out_dispatch<float>(d, tab, nb, max_n, cf, same_rows, rows, s);
}
template <>
void launch_fwd_out<double>(const DecoderDev& d, const Inst<double>* tab, int nb, int max_n, int cf, bool,
                            const int*, hipStream_t s) {
  k_fwd_out_f64<<<dim3((max_n + 15) / 16, nb), 256, 0, s>>>(layer_args(d, d.L - 1), tab);
}

template <typename T>
void launch_filter(const Inst<T>* tab, int nb, int max_n, int add_up, hipStream_t s) {
  const dim3 grid((max_n + FILT_ROWS - 1) / FILT_ROWS, nb);
  k_filter_part<T><<<grid, 256, 0, s>>>(tab);
  k_filter_apply<T><<<grid, 256, 0, s>>>(tab, add_up);
}
template void launch_filter<float>(const Inst<float>*, int, int, int, hipStream_t);
template void launch_filter<double>(const Inst<double>*, int, int, int, hipStream_t);

template <>
void launch_bwd_out<float>(const DecoderDev& d, const Inst<float>* tab, int nb, int max_bblk, hipStream_t s) {
  dim3 grid(max_bblk, nb);
  if (d.prec == PREC_BF16) k_bwd_out<float, __bf16><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab);
  else k_bwd_out<float, float><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab);
}
template <>
void launch_bwd_out<double>(const DecoderDev& d, const Inst<double>* tab, int nb, int max_bblk, hipStream_t s) {
  dim3 grid(max_bblk, nb);
  k_bwd_out<double, double><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab);
}

template <>
void launch_bwd_out_batch<float>(const DecoderDev& d, const Inst<float>* tab, int nb, const int* rows, int nrows,
                                 hipStream_t s) {
  dim3 grid((nrows + BWD_ROWS - 1) / BWD_ROWS, (nb + BWD_NJ - 1) / BWD_NJ);
  if (d.prec == PREC_BF16) k_bwd_out_batch<__bf16><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab, nb, rows, nrows);
  else k_bwd_out_batch<float><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab, nb, rows, nrows);
}
template <>
void launch_bwd_out_batch<double>(const DecoderDev&, const Inst<double>*, int, const int*, int, hipStream_t) {}

template <>
void launch_sums_bwd_out<float>(const DecoderDev& d, const Inst<float>* tab, int nb, int max_entries, int max_sblk,
                                int max_cblk, hipStream_t s) {
  const int n_sum = (max_entries + 15) / 16;
  dim3 grid(n_sum + max_sblk, nb);
  const int m = cubature_merge(nb, max_cblk);
  if (d.prec == PREC_BF16)
    k_sums_bwd_out<float, __bf16><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab, m, n_sum);
  else k_sums_bwd_out<float, float><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab, m, n_sum);
}
template <>
void launch_sums_bwd_out<double>(const DecoderDev& d, const Inst<double>* tab, int nb, int max_entries, int max_sblk,
                                 int max_cblk, hipStream_t s) {
  const int n_sum = (max_entries + 15) / 16;
  dim3 grid(n_sum + max_sblk, nb);
  k_sums_bwd_out<double, double><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab, cubature_merge(nb, max_cblk), n_sum);
}

template <typename T>
void launch_bwd_reduce(const DecoderDev& d, const Inst<T>* tab, int nb, hipStream_t s) {
  const int K = d.wp[d.L - 1];
  k_bwd_reduce<T><<<dim3((K + 15) / 16, nb), 256, 0, s>>>(layer_args(d, d.L - 1), tab);
}
template void launch_bwd_reduce<float>(const DecoderDev&, const Inst<float>*, int, hipStream_t);
template void launch_bwd_reduce<double>(const DecoderDev&, const Inst<double>*, int, hipStream_t);

template <typename T, typename TW, int NCB>
static void bwd_hidden_ib(const DecoderDev& d, int l, const Inst<T>* tab, int nb, bool fd, TileCfg cfg,
                          hipStream_t s) {
  const int tiles = d.wp[l] / 16;
  const int threads = 64 * splitk_waves<T, NCB>::v;
  const LayerArgs la = layer_args(d, l);
  if (fd) {  // the central-difference form: one instance per block
    k_bwd_hidden<T, TW, NCB, 1, true, 1><<<dim3(tiles, nb), threads, 0, s>>>(la, tab, nb);
    return;
  }
  if constexpr (std::is_same<T, float>::value && NCB <= 2) {
    if (cfg.mr == 4) {
      k_bwd_hidden<T, TW, NCB, 4, false, 4><<<dim3(d.wp[l] / 64, (nb + 3) / 4), 256 * tall_ks<TW, NCB, 4>::v, 0, s>>>(la, tab,
                                                                                                            nb);
      return;
    }
    if (cfg.mr == 2) {
      k_bwd_hidden<T, TW, NCB, 4, false, 2><<<dim3(d.wp[l] / 32, (nb + 3) / 4), 256 * tall_ks<TW, NCB, 2>::v, 0, s>>>(la, tab,
                                                                                                            nb);
      return;
    }
  }
  if (cfg.ib == 4) k_bwd_hidden<T, TW, NCB, 4, false, 1><<<dim3(tiles, (nb + 3) / 4), threads, 0, s>>>(la, tab, nb);
  else if (cfg.ib == 2)
    k_bwd_hidden<T, TW, NCB, 2, false, 1><<<dim3(tiles, (nb + 1) / 2), threads, 0, s>>>(la, tab, nb);
  else k_bwd_hidden<T, TW, NCB, 1, false, 1><<<dim3(tiles, nb), threads, 0, s>>>(la, tab, nb);
}

template <typename T, typename TW>
static void bwd_hidden_dispatch(const DecoderDev& d, int l, const Inst<T>* tab, int nb, int cb, bool fd,
                                TileCfg cfg, hipStream_t s) {
  switch (cb / 16) {
    case 1: bwd_hidden_ib<T, TW, 1>(d, l, tab, nb, fd, cfg, s); break;
    case 2: bwd_hidden_ib<T, TW, 2>(d, l, tab, nb, fd, cfg, s); break;
    case 3: bwd_hidden_ib<T, TW, 3>(d, l, tab, nb, fd, cfg, s); break;
    case 4: bwd_hidden_ib<T, TW, 4>(d, l, tab, nb, fd, cfg, s); break;
    default: break;
  }
}

template <>
void launch_bwd_hidden<float>(const DecoderDev& d, int l, const Inst<float>* tab, int nb, int cb, bool fd,
                              TileCfg cfg, hipStream_t s) {
  cfg = resolve(d, l, nb, cb, fd, false, false, cfg);
  if (d.prec == PREC_BF16) bwd_hidden_dispatch<float, __bf16>(d, l, tab, nb, cb, fd, cfg, s);
  else bwd_hidden_dispatch<float, float>(d, l, tab, nb, cb, fd, cfg, s);
}
template <>
void launch_bwd_hidden<double>(const DecoderDev& d, int l, const Inst<double>* tab, int nb, int cb, bool fd,
                               TileCfg, hipStream_t s) {
  bwd_hidden_dispatch<double, double>(d, l, tab, nb, cb, fd, TileCfg{1, 1}, s);
}

template <>
void launch_frame<float>(const DecoderDev& d, const Inst<float>* tab, int nb, int max_n, hipStream_t s) {
  dim3 grid((max_n + 15) / 16, nb);
  if (d.prec == PREC_BF16) k_frame<float, __bf16><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab);
  else k_frame<float, float><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab);
}
template <>
void launch_frame_batch<float>(const DecoderDev& d, const Inst<float>* tab, int nb, int max_n, hipStream_t s) {
  dim3 grid((max_n + 255) / 256, (nb + FRAME_COLS - 1) / FRAME_COLS);
  if (d.prec == PREC_BF16) k_frame_batch<__bf16><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab, nb);
  else k_frame_batch<float><<<grid, 256, 0, s>>>(layer_args(d, d.L - 1), tab, nb);
}
template <>
void launch_frame<double>(const DecoderDev& d, const Inst<double>* tab, int nb, int max_n, hipStream_t s) {
  k_frame<double, double><<<dim3((max_n + 15) / 16, nb), 256, 0, s>>>(layer_args(d, d.L - 1), tab);
}
template <>
void launch_frame_batch<double>(const DecoderDev& d, const Inst<double>* tab, int nb, int max_n, hipStream_t s) {
  launch_frame<double>(d, tab, nb, max_n, s);
}

template <typename T>
void launch_unpack(const Inst<T>* tab, T* u, T* J, T* dJ, T* Hdd, int N, hipStream_t s) {
  k_unpack<T><<<(N + 255) / 256, 256, 0, s>>>(tab, u, J, dJ, Hdd);
}
template void launch_unpack<float>(const Inst<float>*, float*, float*, float*, float*, int, hipStream_t);
template void launch_unpack<double>(const Inst<double>*, double*, double*, double*, double*, int, hipStream_t);

}  // namespace nmr
