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
#include "nmr_internal.h"

#include <type_traits>

namespace nmr {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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

// ---------------------------------------------------------------------------
// One wave computes a 16-row x (NCB*16)-column tile of D = A B with
// A [rows][K] row-major (K contiguous) and B given as Bt [cols][K] (K
// contiguous).  Result: acc[cb][i] = D[4*(lane/16) + i][cb*16 + lane%16].
// K must be a multiple of 32.  B is read through `bload(col, k)` returning
// 4 (or 8) consecutive K entries.
// ---------------------------------------------------------------------------
template <int NCB, typename BL>
__device__ inline void gemm_tile_f32(const float* __restrict__ A, int lda, int K, BL bload,
                                     f32x4 (&acc)[NCB]) {
  const int lane = threadIdx.x & 63;
  const int rA = lane & 15, g = lane >> 4;
  const float* ap = A + (size_t)rA * lda + 4 * g;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const float4 a = *reinterpret_cast<const float4*>(ap + k0);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const float4 b = bload(cb * 16 + rA, k0 + 4 * g);
      acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[cb], 0, 0, 0);
      acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[cb], 0, 0, 0);
      acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc[cb], 0, 0, 0);
      acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc[cb], 0, 0, 0);
    }
  }
}

template <int NCB, typename BL>
__device__ inline void gemm_tile_bf16(const __bf16* __restrict__ A, int lda, int K, BL bload,
                                      f32x4 (&acc)[NCB]) {
  const int lane = threadIdx.x & 63;
  const int rA = lane & 15, g = lane >> 4;
  const __bf16* ap = A + (size_t)rA * lda + 8 * g;
  for (int k0 = 0; k0 < K; k0 += 32) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(ap + k0);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const float4 b0 = bload(cb * 16 + rA, k0 + 8 * g);
      const float4 b1 = bload(cb * 16 + rA, k0 + 8 * g + 4);
      bf16x8 b;
      b[0] = (__bf16)b0.x; b[1] = (__bf16)b0.y; b[2] = (__bf16)b0.z; b[3] = (__bf16)b0.w;
      b[4] = (__bf16)b1.x; b[5] = (__bf16)b1.y; b[6] = (__bf16)b1.z; b[7] = (__bf16)b1.w;
      acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[cb], 0, 0, 0);
    }
  }
}

// Generic tile: MFMA for float / bf16 weights, plain FMA for double.  Writes
// the 16 x (NCB*16) tile into S[col][row] (row stride 17).
template <typename T, typename TW, int NCB, typename BL>
__device__ inline void gemm_tile_to_lds(const TW* __restrict__ A, int lda, int K, BL bload,
                                        T (*S)[17]) {
  const int lane = threadIdx.x & 63;
  if constexpr (std::is_same<TW, double>::value) {
    for (int o = lane; o < NCB * 16 * 16; o += 64) {
      const int c = o >> 4, r = o & 15;
      double acc = 0.0;
      const double* ar = A + (size_t)r * lda;
      for (int k = 0; k < K; k += 4) {
        const double4 b = bload(c, k);
        acc = fma(ar[k], b.x, acc);
        acc = fma(ar[k + 1], b.y, acc);
        acc = fma(ar[k + 2], b.z, acc);
        acc = fma(ar[k + 3], b.w, acc);
      }
      S[c][r] = acc;
    }
  } else {
    f32x4 acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (std::is_same<TW, float>::value)
      gemm_tile_f32<NCB>(A, lda, K, bload, acc);
    else
      gemm_tile_bf16<NCB>(A, lda, K, bload, acc);
    const int rA = lane & 15, g = lane >> 4;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) S[cb * 16 + rA][4 * g + i] = acc[cb][i];
  }
}

template <typename T> struct vec4;
template <> struct vec4<float> { typedef float4 type; };
template <> struct vec4<double> { typedef double4 type; };

// ---------------------------------------------------------------------------
// Forward hidden layer l with the jet activation.  One wave per 16 rows.
// ---------------------------------------------------------------------------
template <typename T, typename TW, int NCB>
__global__ __launch_bounds__(64) void k_fwd_hidden(DecoderDev d, int l, const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  const int m_inp = d.wp[l], m_out = d.w[l + 1], m_outp = d.wp[l + 1];
  const int row0 = blockIdx.x * 16;
  if (row0 >= m_outp) return;
  const int nq = I.n_q;
  const int lane = threadIdx.x;
  const TW* W = reinterpret_cast<const TW*>(d.W[l]) + (size_t)row0 * m_inp;
  const T* bias = reinterpret_cast<const T*>(d.b[l]);
  __shared__ T S[NCB * 16][17];
  __shared__ T sd1[16], sd2[16], sd3[16], sx2[16], sx4[16], sx23[16];
  typedef typename vec4<T>::type V4;

  const T* X = (l & 1) ? I.act0 : I.act1;
  const double* din = I.dec_in;
  auto bload = [&](int c, int k) -> V4 {
    if (l == 0) {
      // input jets: value q, tangents dq (i2) and qdot (i4), unit e_j (i1)
      T v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int kk = k + t;
        T x = T(0);
        if (kk < nq) {
          if (c == 0) x = (T)din[kk];
          else if (c == 1) x = (T)din[nq + kk];
          else if (c == 2) x = (T)din[2 * nq + kk];
          else if (c >= 4 && c < 4 + nq) x = (c - 4 == kk) ? T(1) : T(0);
        }
        v[t] = x;
      }
      return V4{v[0], v[1], v[2], v[3]};
    }
    return *reinterpret_cast<const V4*>(X + (size_t)c * m_inp + k);
  };
  gemm_tile_to_lds<T, TW, NCB>(W, m_inp, m_inp, bload, S);
  __syncthreads();

  T* pre = I.pre[l];
  if (lane < 16) {
    const int row = row0 + lane;
    const bool valid = row < m_out;
    const T x0 = S[0][lane] + (valid ? bias[row] : T(0));
    const T x2 = S[1][lane], x4 = S[2][lane], x23 = S[3][lane];
    T y, d1, d2, d3;
    act_jet(d.act, x0, y, d1, d2, d3);
    sd1[lane] = d1; sd2[lane] = d2; sd3[lane] = d3;
    sx2[lane] = x2; sx4[lane] = x4; sx23[lane] = x23;
    pre[row] = valid ? x0 : T(0);
    S[0][lane] = valid ? y : T(0);
    S[1][lane] = valid ? d1 * x2 : T(0);
    S[2][lane] = valid ? d1 * x4 : T(0);
    S[3][lane] = valid ? d1 * x23 + d2 * x2 * x2 : T(0);
  }
  __syncthreads();
  for (int p = lane; p < 16 * nq; p += 64) {
    const int r = p & 15, j = p >> 4;
    const bool valid = row0 + r < m_out;
    const T x1 = S[4 + j][r], x12 = S[4 + nq + j][r], x14 = S[4 + 2 * nq + j][r],
            x123 = S[4 + 3 * nq + j][r];
    const T d1 = sd1[r], d2 = sd2[r], d3 = sd3[r], x2 = sx2[r], x4 = sx4[r], x23 = sx23[r];
    pre[(size_t)(1 + j) * m_outp + row0 + r] = valid ? x1 : T(0);
    S[4 + j][r] = valid ? d1 * x1 : T(0);
    S[4 + nq + j][r] = valid ? d1 * x12 + d2 * x1 * x2 : T(0);
    S[4 + 2 * nq + j][r] = valid ? d1 * x14 + d2 * x1 * x4 : T(0);
    S[4 + 3 * nq + j][r] = valid ? d1 * x123 + d2 * (x1 * x23 + T(2) * x2 * x12) + d3 * x1 * x2 * x2 : T(0);
  }
  __syncthreads();
  if (l + 2 < d.L) {
    T* out = (l & 1) ? I.act1 : I.act0;
    const int C = 4 + 4 * nq;
    for (int p = lane; p < C * 16; p += 64) {
      const int c = p >> 4, r = p & 15;
      out[(size_t)c * m_outp + row0 + r] = S[c][r];
    }
  } else {
    // last hidden layer: fold into the output channels (the output layer is
    // linear, so eq. delta_j can be combined before it)
    const T dt = (T)I.dt;
    const int C = 2 + 2 * nq;
    for (int p = lane; p < C * 16; p += 64) {
      const int c = p >> 4, r = p & 15;
      T v;
      if (c == 0) v = S[0][r];
      else if (c <= nq) v = S[4 + c - 1][r];
      else if (c <= 2 * nq) {
        const int j = c - 1 - nq;
        v = S[4 + 3 * nq + j][r] + T(3) * S[4 + nq + j][r] - dt * S[4 + 2 * nq + j][r];
      } else v = S[3][r];
      I.fold[(size_t)c * m_outp + row0 + r] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Output layer: rec[i][c] = keep_i (W_L fold + b_L e_0)[i][c].  4 waves per
// block, each wave RT tiles of 16 rows; the folded activations are staged in
// LDS once per block.
// ---------------------------------------------------------------------------
template <typename T, typename TW, int NCB, int RT>
__global__ __launch_bounds__(256) void k_fwd_out(DecoderDev d, const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  const int l = d.L - 1;
  const int K = d.wp[l];
  const int rows_per_blk = 4 * 16 * RT;
  const int blk_row0 = blockIdx.x * rows_per_blk;
  if (blk_row0 >= I.N) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* F = reinterpret_cast<T*>(smem_raw);  // [NCB*16][K + 4]
  const int ldf = K + 4;
  for (int p = threadIdx.x; p < NCB * 16 * K; p += 256) {
    const int c = p / K, k = p - c * K;
    F[c * ldf + k] = I.fold[(size_t)c * K + k];
  }
  __syncthreads();
  typedef typename vec4<T>::type V4;
  auto bload = [&](int c, int k) -> V4 { return *reinterpret_cast<const V4*>(F + c * ldf + k); };
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const TW* W = reinterpret_cast<const TW*>(d.W[l]);
  const T* bias = reinterpret_cast<const T*>(d.b[l]);
  __shared__ T S[4][NCB * 16][17];
  const int Cf = I.Cf;
  for (int t = 0; t < RT; ++t) {
    const int row0 = blk_row0 + (t * 4 + wave) * 16;
    if (row0 < I.N) {
      gemm_tile_to_lds<T, TW, NCB>(W + (size_t)row0 * K, K, K, bload, S[wave]);
    }
    __syncthreads();
    if (row0 < I.N) {
      for (int p = lane; p < 16 * Cf; p += 64) {
        const int r = p / Cf, c = p - r * Cf;
        const int row = row0 + r;
        if (row < I.N) {
          T v = S[wave][c][r] + (c == 0 ? bias[row] : T(0));
          I.rec[(size_t)row * Cf + c] = v * I.keep[row];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Filter (I - U U^T) of every output channel and u += U p (n_p > 0 only).
// One block per instance.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_filter(const Inst<T>* __restrict__ tab, int add_up) {
  const Inst<T>& I = tab[blockIdx.y];
  const int np = I.n_p, Cf = I.Cf, N = I.N;
  if (np == 0) return;
  __shared__ double Y[NMR_MAX_R][64];  // U^T rec, n_p x Cf (Cf <= 64)
  __shared__ double pv[NMR_MAX_R];
  for (int e = threadIdx.x; e < np * Cf; e += 256) {
    const int k = e / Cf, c = e - k * Cf;
    double acc = 0.0;
    for (int i = 0; i < N; ++i) acc += (double)I.U[(size_t)i * np + k] * (double)I.rec[(size_t)i * Cf + c];
    Y[k][c] = acc;
  }
  if (threadIdx.x < np) pv[threadIdx.x] = I.r[threadIdx.x];
  __syncthreads();
  for (int e = threadIdx.x; e < N * Cf; e += 256) {
    const int i = e / Cf, c = e - i * Cf;
    double v = (double)I.rec[e];
    for (int k = 0; k < np; ++k) v -= (double)I.U[(size_t)i * np + k] * Y[k][c];
    if (c == 0 && add_up)
      for (int k = 0; k < np; ++k) v += (double)I.U[(size_t)i * np + k] * pv[k];
    I.rec[e] = (T)v;
  }
}

// ---------------------------------------------------------------------------
// Backward through the output layer: partial sums of W_L^T s over row chunks.
// s_i = seed_i - sum_k U_ik (U^T P a)_k (the filter's transpose).
// ---------------------------------------------------------------------------
#define BWD_ROWS 128
__device__ inline double wval(double w) { return w; }
__device__ inline double wval(float w) { return (double)w; }
__device__ inline double wval(__bf16 w) { return (double)(float)w; }
template <typename T, typename TW>
__global__ __launch_bounds__(256) void k_bwd_out(DecoderDev d, const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  if ((int)blockIdx.x >= I.n_bblk) return;
  const int l = d.L - 1;
  const int K = d.wp[l];
  const int i0 = blockIdx.x * BWD_ROWS;
  const int i1 = min(i0 + BWD_ROWS, I.N);
  __shared__ double s[BWD_ROWS];
  const int np = I.n_p;
  const double* uta = I.sum_mass + I.R * I.R + I.R * I.n_q + I.R;
  for (int i = i0 + threadIdx.x; i < i1; i += 256) {
    double v = (double)I.seed[i];
    for (int k = 0; k < np; ++k) v -= (double)I.U[(size_t)i * np + k] * uta[k];
    s[i - i0] = v;
  }
  __syncthreads();
  const TW* W = reinterpret_cast<const TW*>(d.W[l]);
  for (int k = threadIdx.x; k < K; k += 256) {
    double acc = 0.0;
    for (int i = i0; i < i1; ++i) acc = fma(wval(W[(size_t)i * K + k]), s[i - i0], acc);
    I.part_bwd[(size_t)blockIdx.x * K + k] = acc;
  }
}

// ---------------------------------------------------------------------------
// Sum the output-layer partials (fixed order) and apply sigma' of the last
// hidden layer: xb0 = s1 zb0, xb1_j = s2 x1_j zb0 (the seed is real).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_reduce(DecoderDev d, const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  const int l = d.L - 1;  // output layer; its input is hidden layer l-1
  const int K = d.wp[l];
  const int kk = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + kk;
  __shared__ double part[4][64];
  double acc = 0.0;
  if (k < K)
    for (int b = sl; b < I.n_bblk; b += 4) acc += I.part_bwd[(size_t)b * K + k];
  part[sl][kk] = acc;
  __syncthreads();
  if (sl == 0 && k < K) {
    const double zb0 = ((part[0][kk] + part[1][kk]) + part[2][kk]) + part[3][kk];
    const T* pre = I.pre[l - 1];
    const T x0 = pre[k];
    T d1, d2;
    act_d12(d.act, x0, d1, d2);
    T* xb = I.zb0;
    xb[k] = (k < d.w[l]) ? (T)(d1 * zb0) : T(0);
    for (int j = 0; j < I.n_q; ++j)
      xb[(size_t)(1 + j) * K + k] = (k < d.w[l]) ? (T)(d2 * pre[(size_t)(1 + j) * K + k] * zb0) : T(0);
  }
}

// ---------------------------------------------------------------------------
// Backward through hidden layer l: zb_prev = W_l^T xb_l (a GEMM with the
// transposed weights stored row-major), then either sigma' of layer l-1 or,
// at the input, J^T a and a . H.
// ---------------------------------------------------------------------------
template <typename T, typename TW, int NCB>
__global__ __launch_bounds__(64) void k_bwd_hidden(DecoderDev d, const void* WT_, int l,
                                                   const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  const int K = d.wp[l + 1];     // reduction over the outputs of layer l
  const int m_in = d.w[l], m_inp = d.wp[l];
  const int row0 = blockIdx.x * 16;
  if (row0 >= m_inp) return;
  const int nq = I.n_q;
  const int lane = threadIdx.x;
  const int step = d.L - 2 - l;  // 0 for the last hidden layer
  const T* xb = (step & 1) ? I.zb1 : I.zb0;
  T* xb_out = (step & 1) ? I.zb0 : I.zb1;
  const TW* WT = reinterpret_cast<const TW*>(WT_) + (size_t)row0 * K;
  __shared__ T S[NCB * 16][17];
  typedef typename vec4<T>::type V4;
  auto bload = [&](int c, int k) -> V4 {
    return *reinterpret_cast<const V4*>(xb + (size_t)c * K + k);
  };
  gemm_tile_to_lds<T, TW, NCB>(WT, K, K, bload, S);
  __syncthreads();
  if (l > 0) {
    const T* pre = I.pre[l - 1];
    for (int p = lane; p < 16 * (1 + nq); p += 64) {
      const int r = p & 15, c = p >> 4;
      const int row = row0 + r;
      const T x0 = pre[row];
      T d1, d2;
      act_d12(d.act, x0, d1, d2);
      T v;
      if (c == 0) v = d1 * S[0][r];
      else v = d1 * S[c][r] + d2 * pre[(size_t)c * m_inp + row] * S[0][r];
      xb_out[(size_t)c * m_inp + row] = (row < m_in) ? v : T(0);
    }
  } else {
    for (int p = lane; p < 16 * (1 + nq); p += 64) {
      const int r = p & 15, c = p >> 4;
      const int row = row0 + r;
      if (row < nq) {
        if (c == 0) I.JTa[row] = (double)S[0][r];
        else I.Bq[(size_t)row * nq + (c - 1)] = (double)S[c][r];
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
// launchers
// ---------------------------------------------------------------------------
template <typename T, typename TW>
static void fwd_hidden_dispatch(const DecoderDev& d, int l, const Inst<T>* tab, int nb, int cp, hipStream_t s) {
  dim3 grid(d.wp[l + 1] / 16, nb);
  switch (cp / 16) {
    case 1: k_fwd_hidden<T, TW, 1><<<grid, 64, 0, s>>>(d, l, tab); break;
    case 2: k_fwd_hidden<T, TW, 2><<<grid, 64, 0, s>>>(d, l, tab); break;
    case 3: k_fwd_hidden<T, TW, 3><<<grid, 64, 0, s>>>(d, l, tab); break;
    case 4: k_fwd_hidden<T, TW, 4><<<grid, 64, 0, s>>>(d, l, tab); break;
    case 5: k_fwd_hidden<T, TW, 5><<<grid, 64, 0, s>>>(d, l, tab); break;
    case 6: k_fwd_hidden<T, TW, 6><<<grid, 64, 0, s>>>(d, l, tab); break;
    case 7: k_fwd_hidden<T, TW, 7><<<grid, 64, 0, s>>>(d, l, tab); break;
    case 8: k_fwd_hidden<T, TW, 8><<<grid, 64, 0, s>>>(d, l, tab); break;
    default: break;
  }
}

template <>
void launch_fwd_hidden<float>(const DecoderDev& d, int l, const Inst<float>* tab, int nb, int cp, hipStream_t s) {
  if (d.prec == PREC_BF16) fwd_hidden_dispatch<float, __bf16>(d, l, tab, nb, cp, s);
  else fwd_hidden_dispatch<float, float>(d, l, tab, nb, cp, s);
}
template <>
void launch_fwd_hidden<double>(const DecoderDev& d, int l, const Inst<double>* tab, int nb, int cp, hipStream_t s) {
  fwd_hidden_dispatch<double, double>(d, l, tab, nb, cp, s);
}

template <typename T, typename TW>
static void fwd_out_dispatch(const DecoderDev& d, const Inst<T>* tab, int nb, int max_n, int cf, hipStream_t s) {
  constexpr int RT = 2;
  const int rows = 4 * 16 * RT;
  dim3 grid((max_n + rows - 1) / rows, nb);
  const int K = d.wp[d.L - 1];
  const size_t lds = (size_t)cf * (K + 4) * sizeof(T);
  switch (cf / 16) {
    case 1: k_fwd_out<T, TW, 1, RT><<<grid, 256, lds, s>>>(d, tab); break;
    case 2: k_fwd_out<T, TW, 2, RT><<<grid, 256, lds, s>>>(d, tab); break;
    case 3: k_fwd_out<T, TW, 3, RT><<<grid, 256, lds, s>>>(d, tab); break;
    case 4: k_fwd_out<T, TW, 4, RT><<<grid, 256, lds, s>>>(d, tab); break;
    default: break;
  }
}

template <>
void launch_fwd_out<float>(const DecoderDev& d, const Inst<float>* tab, int nb, int max_n, int cf, hipStream_t s) {
  if (d.prec == PREC_BF16) fwd_out_dispatch<float, __bf16>(d, tab, nb, max_n, cf, s);
  else fwd_out_dispatch<float, float>(d, tab, nb, max_n, cf, s);
}
template <>
void launch_fwd_out<double>(const DecoderDev& d, const Inst<double>* tab, int nb, int max_n, int cf, hipStream_t s) {
  fwd_out_dispatch<double, double>(d, tab, nb, max_n, cf, s);
}

template <typename T>
void launch_filter(const Inst<T>* tab, int nb, int add_up, hipStream_t s) {
  k_filter<T><<<dim3(1, nb), 256, 0, s>>>(tab, add_up);
}
template void launch_filter<float>(const Inst<float>*, int, int, hipStream_t);
template void launch_filter<double>(const Inst<double>*, int, int, hipStream_t);

template <>
void launch_bwd_out<float>(const DecoderDev& d, const Inst<float>* tab, int nb, int max_bblk, hipStream_t s) {
  dim3 grid(max_bblk, nb);
  if (d.prec == PREC_BF16) k_bwd_out<float, __bf16><<<grid, 256, 0, s>>>(d, tab);
  else k_bwd_out<float, float><<<grid, 256, 0, s>>>(d, tab);
}
template <>
void launch_bwd_out<double>(const DecoderDev& d, const Inst<double>* tab, int nb, int max_bblk, hipStream_t s) {
  dim3 grid(max_bblk, nb);
  k_bwd_out<double, double><<<grid, 256, 0, s>>>(d, tab);
}

template <typename T>
void launch_bwd_reduce(const DecoderDev& d, const Inst<T>* tab, int nb, hipStream_t s) {
  const int K = d.wp[d.L - 1];
  k_bwd_reduce<T><<<dim3((K + 63) / 64, nb), 256, 0, s>>>(d, tab);
}
template void launch_bwd_reduce<float>(const DecoderDev&, const Inst<float>*, int, hipStream_t);
template void launch_bwd_reduce<double>(const DecoderDev&, const Inst<double>*, int, hipStream_t);

template <typename T, typename TW>
static void bwd_hidden_dispatch(const DecoderDev& d, const void* WT, int l, const Inst<T>* tab, int nb, int cb,
                                hipStream_t s) {
  dim3 grid(d.wp[l] / 16, nb);
  switch (cb / 16) {
    case 1: k_bwd_hidden<T, TW, 1><<<grid, 64, 0, s>>>(d, WT, l, tab); break;
    case 2: k_bwd_hidden<T, TW, 2><<<grid, 64, 0, s>>>(d, WT, l, tab); break;
    case 3: k_bwd_hidden<T, TW, 3><<<grid, 64, 0, s>>>(d, WT, l, tab); break;
    case 4: k_bwd_hidden<T, TW, 4><<<grid, 64, 0, s>>>(d, WT, l, tab); break;
    default: break;
  }
}

template <>
void launch_bwd_hidden<float>(const DecoderDev& d, int l, const Inst<float>* tab, int nb, int cb, hipStream_t s) {
  if (d.prec == PREC_BF16) bwd_hidden_dispatch<float, __bf16>(d, d.WT[l], l, tab, nb, cb, s);
  else bwd_hidden_dispatch<float, float>(d, d.WT[l], l, tab, nb, cb, s);
}
template <>
void launch_bwd_hidden<double>(const DecoderDev& d, int l, const Inst<double>* tab, int nb, int cb, hipStream_t s) {
  bwd_hidden_dispatch<double, double>(d, d.WT[l], l, tab, nb, cb, s);
}

template <typename T>
void launch_unpack(const Inst<T>* tab, T* u, T* J, T* dJ, T* Hdd, int N, hipStream_t s) {
  k_unpack<T><<<(N + 255) / 256, 256, 0, s>>>(tab, u, J, dJ, Hdd);
}
template void launch_unpack<float>(const Inst<float>*, float*, float*, float*, float*, int, hipStream_t);
template void launch_unpack<double>(const Inst<double>*, double*, double*, double*, double*, int, hipStream_t);

}  // namespace nmr
