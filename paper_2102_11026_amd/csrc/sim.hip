// Simulation kernels: rest shape and lumped mass (Sec. 3.1), cubature
// weights (Sec. 5.2), cubature force and reduced stiffness of neo-Hookean
// tets (Sec. 5), the mass terms of the reduced residual and Newton matrix
// (eq. our_equation_of_motion, eq. system_mat), fixed-order partial sums and
// the FP64 LU solve and state update (Sec. 3.2).
//
// Every cross-block sum is written as per-block partials and added in a
// fixed order, so a run is bitwise reproducible and an instance gives the
// same result alone or inside a batch.
#include "nmr_internal.h"

namespace nmr {

// ---------------------------------------------------------------------------
// setup: B_m = D_m^-1 and V_e of cubature tets, volumes of all tets, then the
// lumped mass m_v = sum over incident tets of rho V_e / 4 (vertex -> tet CSR,
// fixed order).
// ---------------------------------------------------------------------------
__device__ inline void edge_matrix(const double* X, const int* t, double D[3][3]) {
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < 3; ++i) D[i][c] = X[3 * t[c + 1] + i] - X[3 * t[0] + i];
}

__device__ inline double det3(const double D[3][3]) {
  return D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) - D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
         D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
}

__global__ void k_tet_volume(const double* X, const int* tets, int m, double* Ve) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  double D[3][3];
  edge_matrix(X, tets + 4 * e, D);
  Ve[e] = det3(D) / 6.0;
}

template <typename T>
__global__ void k_cub_rest(const double* X, const int* tets, const int* cub_ids, int n_cub, T* Bm, T* Ve) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_cub) return;
  double D[3][3];
  edge_matrix(X, tets + 4 * cub_ids[s], D);
  const double det = det3(D);
  const double inv = 1.0 / det;
  double B[3][3];
  B[0][0] = (D[1][1] * D[2][2] - D[1][2] * D[2][1]) * inv;
  B[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * inv;
  B[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * inv;
  B[1][0] = (D[1][2] * D[2][0] - D[1][0] * D[2][2]) * inv;
  B[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * inv;
  B[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * inv;
  B[2][0] = (D[1][0] * D[2][1] - D[1][1] * D[2][0]) * inv;
  B[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * inv;
  B[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * inv;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Bm[9 * s + 3 * i + j] = (T)B[i][j];
  Ve[s] = (T)(det / 6.0);
}

template <typename T>
__global__ void k_lumped_mass(const int* vt_ptr, const int* vt_ent, const double* Ve, int n, double rho, T* mass) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double m = 0.0;
  for (int p = vt_ptr[v]; p < vt_ptr[v + 1]; ++p) m += rho * Ve[vt_ent[p]] * 0.25;
  for (int c = 0; c < 3; ++c) mass[3 * v + c] = (T)m;
}

template <typename T>
void launch_rest_shape(const double* X, const int* tets, int m, const int* cub_ids, int n_cub, const int* vt_ptr,
                       const int* vt_ent, int n, double rho, T* cub_Bm, T* cub_Ve, T* mass, double* Ve_tmp,
                       hipStream_t s) {
  k_tet_volume<<<(m + 255) / 256, 256, 0, s>>>(X, tets, m, Ve_tmp);
  k_cub_rest<T><<<(n_cub + 255) / 256, 256, 0, s>>>(X, tets, cub_ids, n_cub, cub_Bm, cub_Ve);
  k_lumped_mass<T><<<(n + 255) / 256, 256, 0, s>>>(vt_ptr, vt_ent, Ve_tmp, n, rho, mass);
}
template void launch_rest_shape<float>(const double*, const int*, int, const int*, int, const int*, const int*, int,
                                       double, float*, float*, float*, double*, hipStream_t);
template void launch_rest_shape<double>(const double*, const int*, int, const int*, int, const int*, const int*, int,
                                        double, double*, double*, double*, double*, hipStream_t);


// ---------------------------------------------------------------------------
// step begin: cubature weights from the weight net at rbar (softplus after
// every layer, scaled), the Newton start r = rbar and the decoder input.
// mode BEGIN_SYSTEM keeps r and only refreshes weights and decoder input.
// Every block recomputes the small hidden layers of the weight net and then
// produces 256 of the |C| outputs.
// ---------------------------------------------------------------------------
__device__ inline double softplus(double x) { return x > 0.0 ? x + log1p(exp(-x)) : log1p(exp(x)); }

template <typename T>
__device__ inline double dot_unrolled(const T* __restrict__ w, const double* __restrict__ z, int n) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int k = 0;
  for (; k + 4 <= n; k += 4) {
    a0 += (double)ldg<T>(w + k) * z[k];
    a1 += (double)ldg<T>(w + k + 1) * z[k + 1];
    a2 += (double)ldg<T>(w + k + 2) * z[k + 2];
    a3 += (double)ldg<T>(w + k + 3) * z[k + 3];
  }
  for (; k < n; ++k) a0 += (double)ldg<T>(w + k) * z[k];
  return (a0 + a1) + (a2 + a3);
}

#define WN_MAXW 1024
template <typename T>
__global__ __launch_bounds__(256) void k_step_begin(const Inst<T>* __restrict__ tab, int mode) {
  const Inst<T>& I = tab[blockIdx.y];
  load_now(I.active, I.R, I.n_p, I.n_q, I.rbar, I.r, I.rdot, I.dec_in, I.wn_L, I.wn_scale, I.cub_w);
  if (!I.active) return;
  const int R = I.R, np = I.n_p, nq = I.n_q;
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < nq; k += 256) {
      const double rb = ldg<double>(I.rbar + np + k), rc = ldg<double>(I.r + np + k);
      const double rd = ldg<double>(I.rdot + np + k);
      const double q = (mode == BEGIN_STEP) ? rb : rc;
      stg<double>(I.dec_in + k, q);
      stg<double>(I.dec_in + nq + k, q - rb);
      stg<double>(I.dec_in + 2 * nq + k, rd);
    }
    if (mode == BEGIN_STEP)
      for (int k = threadIdx.x; k < R; k += 256) stg<double>(I.r + k, ldg<double>(I.rbar + k));
  }
  if (I.wn_L == 0) return;
  const int last = I.wn_L - 1;
  const int o0 = blockIdx.x * 256;
  if (o0 >= I.wn_w[I.wn_L]) return;
  __shared__ double z[2][WN_MAXW];
  for (int k = threadIdx.x; k < I.wn_w[0]; k += 256) z[0][k] = ldg<double>(I.rbar + k);
  __syncthreads();
  for (int l = 0; l < last; ++l) {
    const double* in = z[l & 1];
    double* out = z[(l + 1) & 1];
    const int wi = I.wn_w[l], wo = I.wn_w[l + 1];
    for (int o = threadIdx.x; o < wo; o += 256)
      out[o] = softplus((double)ldg<T>(I.wn_b[l] + o) + dot_unrolled(I.wn_W[l] + (size_t)o * wi, in, wi));
    __syncthreads();
  }
  const double* in = z[last & 1];
  const int wi = I.wn_w[last], wo = I.wn_w[last + 1];
  const int o = o0 + threadIdx.x;
  if (o < wo)
    stg<T>(I.cub_w + o, (T)(I.wn_scale * softplus((double)ldg<T>(I.wn_b[last] + o) +
                                                   dot_unrolled(I.wn_W[last] + (size_t)o * wi, in, wi))));
}

template <typename T>
void launch_step_begin(const Inst<T>* tab, int nb, int mode, int max_cub, hipStream_t s) {
  k_step_begin<T><<<dim3((max_cub + 255) / 256, nb), 256, 0, s>>>(tab, mode);
}
template void launch_step_begin<float>(const Inst<float>*, int, int, int, hipStream_t);
template void launch_step_begin<double>(const Inst<double>*, int, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Cubature: a block of 4 cubature tets (times the merge factor m) is split
// over 4 "virtual waves", virtual wave v taking the tets e0 + v + 4k.  A
// virtual wave is a real wave of a 4-wave block (W = 4: one tet per wave at a
// time, the latency-bound form of small launches) or a 16-lane group of a
// 1-wave block (W = 1: four tets per wave at once, the throughput form of
// large launches with R <= 16).  Per tet e with deformation gradient
// F = D_s B_m, first Piola stress P and its tangent dP:
//   dF_r = dF/dr_r = sum_a Jt_{a,r} (x) g_a,   g_a = gradient of hat fn a,
//   fr_r += w V P : dF_r,   Kr_rs += w V dP[dF_r] : dF_s,
//   f_a   = w V P g_a (element force, gathered per DOF later),
// which equals Jt_e^T f_e and Jt_e^T K_e Jt_e without forming the 12 x 12
// K_e.  Neo-Hookean: P = mu (F - F^-T) + lam ln J F^-T,
//   dP[dF] = mu dF + (mu - lam ln J) F^-T dF^T F^-T + lam tr(F^-1 dF) F^-T.
// F and P are computed by every lane of a tet's lane group, dF_r and dP[dF_r]
// by its lane r, the stiffness blocks by all 64 lanes of the wave.  Element
// math in T, accumulation in FP64, one accumulator set per virtual wave, the
// virtual waves' sums added in order: both forms give the same bits.
// Launches of many instances or of a large mesh merge m = cubature_merge(nb,
// max_cblk) consecutive blocks of tets into one (partial b then covers blocks
// b m .. b m + m - 1).
// ---------------------------------------------------------------------------
#define CUB_VWAVES 4

template <typename T, int RB, int W>
__device__ __forceinline__ void cubature_block(const Inst<T>* __restrict__ tab, int bx, int by, int m) {
  constexpr int G = CUB_VWAVES / W;  // tets per wave at once (lane groups)
  constexpr int LG = 64 / G;         // lanes per group
  static_assert(G == 1 || RB <= LG, "a lane group must hold R lanes");
  const Inst<T>& I = tab[by];
  load_now(I.active, I.n_cblk, I.R, I.cu_na, I.mu, I.lam, I.cub_per_blk, I.n_cub, I.cub_v, I.cub_Bm, I.cu_w, I.cub_Ve,
           I.X, I.cu_u, I.cu_u_ld, I.cu_Ja, I.cu_Ja_ld, I.cu_Jb, I.cu_Jb_ld, I.status, I.fe, I.part_cub);
  if (!I.active) return;
  if (bx * m >= I.n_cblk) return;
  const int R = I.R;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = lane / LG, gl = lane % LG;  // lane group (tet of the round) and lane within it
  const int na = I.cu_na;
  const T mu = (T)I.mu, lam = (T)I.lam;
  __shared__ T xs[W][G][12];
  __shared__ T J12[W][G][12][RB + 1];
  __shared__ T dFs[W][G][RB][9];
  __shared__ T dPs[W][G][RB][9];
  __shared__ T sw[W][G];     // w V of the round's tets
  __shared__ int sok[W][G];  // 1: the group's tet is in the range
  __shared__ double sfa[W][64];
  __shared__ double red[RB * RB + RB];
  // the R x R stiffness sums in BS x BS blocks (BS = 2, or 4 when R > 16:
  // fewer LDS reads per entry): lane l owns blocks l + 64 t, block b covering
  // rows BS (b / nbs) + [0, BS) and columns BS (b % nbs) + [0, BS) (each entry
  // the same 9-term dot product in the same order as unblocked)
  constexpr int BS = RB > 16 ? 4 : 2;
  constexpr int BT = ((RB + BS - 1) / BS * ((RB + BS - 1) / BS) + 63) / 64;
  const int nbs = (R + BS - 1) / BS;
  double kacc[G][BT][BS * BS];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int t = 0; t < BT; ++t)
#pragma unroll
      for (int q = 0; q < BS * BS; ++q) kacc[g][t][q] = 0.0;
  double facc = 0.0;
  const int e0 = bx * m * I.cub_per_blk;
  const int e1 = min(e0 + m * I.cub_per_blk, I.n_cub);
  constexpr int JT = (12 * RB + LG - 1) / LG;
  // first round trip of tet e: its vertices, B_m, weight and volume (none
  // depends on another load)
  auto load_r1 = [&](int e, int4& tv, T (&Bmv)[9], T& wV) {
    tv = ldg<int4>(I.cub_v + 4 * e);
#pragma unroll
    for (int q = 0; q < 9; ++q) Bmv[q] = ldg<T>(I.cub_Bm + 9 * e + q);
    wV = ldg<T>(I.cu_w + e) * ldg<T>(I.cub_Ve + e);
  };
  // second round trip: positions and Jacobian rows of the 12 DOFs, every
  // load from an index clamped into range
  auto load_r2 = [&](const int4& tv, T& xv, T (&jv)[JT]) {
    auto dof_of = [&](int ac) {
      const int a = ac / 3;
      const int v = a == 0 ? tv.x : a == 1 ? tv.y : a == 2 ? tv.z : tv.w;
      return 3 * v + (ac - 3 * a);
    };
    const int dx = dof_of(min(gl, 11));
    xv = ldg<T>(I.X + dx) + ldg<T>(I.cu_u + (size_t)dx * I.cu_u_ld);
#pragma unroll
    for (int t = 0; t < JT; ++t) {
      const int p = min(gl + LG * t, 12 * R - 1);
      const int ac = p / R, r = p - ac * R;
      const int dof = dof_of(ac);
      const T* src = (r < na) ? I.cu_Ja + (size_t)dof * I.cu_Ja_ld + r : I.cu_Jb + (size_t)dof * I.cu_Jb_ld + (r - na);
      jv[t] = ldg<T>(src);
    }
  };
  // this wave's LDS writes are visible to its own reads (outstanding global
  // loads, the prefetches of the next tets, stay in flight)
  auto lds_fence = []() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
  };
  // the round's G tets from their loaded operands (ok: this lane's tet is in range)
  auto tets = [&](int e, bool ok, const T (&Bmv)[9], const T wV, const T xv, const T (&jv)[JT]) {
    if (gl < 12) xs[wave][grp][gl] = xv;
#pragma unroll
    for (int t = 0; t < JT; ++t) {
      const int p = gl + LG * t;
      if (p < 12 * R) {
        const int ac = p / R, r = p - ac * R;
        J12[wave][grp][ac][r] = jv[t];
      }
    }
    if (gl == 0) {
      sw[wave][grp] = wV;
      sok[wave][grp] = ok ? 1 : 0;
    }
    lds_fence();
    T G3[4][3];
    for (int j = 0; j < 3; ++j) {
      G3[1][j] = Bmv[0 * 3 + j];
      G3[2][j] = Bmv[1 * 3 + j];
      G3[3][j] = Bmv[2 * 3 + j];
      G3[0][j] = -(G3[1][j] + G3[2][j] + G3[3][j]);
    }
    T F[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T acc = T(0);
        for (int a = 1; a < 4; ++a) acc += (xs[wave][grp][3 * a + i] - xs[wave][grp][i]) * G3[a][j];
        F[i][j] = acc;
      }
    const T det = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                  F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
    if (ok && det <= T(0) && gl == 0) atomicOr(I.status, ST_INVERTED);
    const T id = T(1) / det;
    T A[3][3];  // F^-T
    A[0][0] = (F[1][1] * F[2][2] - F[1][2] * F[2][1]) * id;
    A[1][0] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * id;
    A[2][0] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * id;
    A[0][1] = (F[1][2] * F[2][0] - F[1][0] * F[2][2]) * id;
    A[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * id;
    A[2][1] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * id;
    A[0][2] = (F[1][0] * F[2][1] - F[1][1] * F[2][0]) * id;
    A[1][2] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * id;
    A[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * id;
    const T lnJ = log(det);
    T P[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) P[i][j] = mu * (F[i][j] - A[i][j]) + lam * lnJ * A[i][j];
    const T c2 = mu - lam * lnJ;
    if (gl < R) {
      const int r = gl;
      T dF[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          T acc = T(0);
          for (int a = 0; a < 4; ++a) acc += J12[wave][grp][3 * a + i][r] * G3[a][j];
          dF[i][j] = acc;
        }
      T tr = T(0);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) tr += A[i][j] * dF[i][j];
      T M[3][3];  // dF^T A
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = dF[0][i] * A[0][j] + dF[1][i] * A[1][j] + dF[2][i] * A[2][j];
      T fr = T(0);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          const T ADA = A[i][0] * M[0][j] + A[i][1] * M[1][j] + A[i][2] * M[2][j];
          dPs[wave][grp][r][3 * i + j] = mu * dF[i][j] + c2 * ADA + lam * tr * A[i][j];
          dFs[wave][grp][r][3 * i + j] = dF[i][j];
          fr += P[i][j] * dF[i][j];
        }
      if (ok) facc += (double)wV * (double)fr;
    }
    if (ok && gl < 12) {
      const int a = gl / 3, i = gl % 3;
      T f = T(0);
      for (int j = 0; j < 3; ++j) f += P[i][j] * G3[a][j];
      stg<T>(I.fe + (size_t)e * 12 + gl, wV * f);
    }
    lds_fence();
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (!sok[wave][g]) continue;
      const double wg = (double)sw[wave][g];
#pragma unroll
      for (int t = 0; t < BT; ++t) {
        const int b = lane + 64 * t;
        if (b < nbs * nbs) {
          const int r0 = BS * (b / nbs), s0 = BS * (b % nbs);
          int rr[BS], ss[BS];
#pragma unroll
          for (int i = 0; i < BS; ++i) {
            rr[i] = min(r0 + i, R - 1);
            ss[i] = min(s0 + i, R - 1);
          }
          T a[BS][BS];
#pragma unroll
          for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int j = 0; j < BS; ++j) a[i][j] = T(0);
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            T pv[BS], fv[BS];
#pragma unroll
            for (int i = 0; i < BS; ++i) {
              pv[i] = dPs[wave][g][rr[i]][k];
              fv[i] = dFs[wave][g][ss[i]][k];
            }
#pragma unroll
            for (int i = 0; i < BS; ++i)
#pragma unroll
              for (int j = 0; j < BS; ++j) a[i][j] += pv[i] * fv[j];
          }
#pragma unroll
          for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int j = 0; j < BS; ++j) kacc[g][t][BS * i + j] += wg * (double)a[i][j];
        }
      }
    }
    lds_fence();
  };
  // round k of this wave covers tets eb + 4 k .. eb + 4 k + G - 1
  constexpr int S = CUB_VWAVES;
  int eb = e0 + wave * G;
  if (e1 - e0 <= S) {
    // one round: nothing to overlap
    if (eb < e1) {
      const int e = min(eb + grp, e1 - 1);
      int4 tv;
      T Bmv[9], wV, xv, jv[JT];
      load_r1(e, tv, Bmv, wV);
      load_r2(tv, xv, jv);
      tets(e, eb + grp < e1, Bmv, wV, xv, jv);
    }
  } else if (eb < e1) {
    // three-stage pipeline: while round k is computed, the second round trip
    // of round k + 1 and the first of round k + 2 are in flight (indices
    // clamped to the last tet of the range; past it the loads go unused)
    int4 tv1, tv2;
    T Bm0[9], Bm1[9], Bm2[9], wV0, wV1, wV2, xv0, xv1, jv0[JT], jv1[JT];
    load_r1(min(eb + grp, e1 - 1), tv2, Bm0, wV0);
    load_r1(min(eb + S + grp, e1 - 1), tv1, Bm1, wV1);
    load_r2(tv2, xv0, jv0);
    for (; eb < e1; eb += S) {
      load_r1(min(eb + 2 * S + grp, e1 - 1), tv2, Bm2, wV2);
      load_r2(tv1, xv1, jv1);
      tets(min(eb + grp, e1 - 1), eb + grp < e1, Bm0, wV0, xv0, jv0);
      tv1 = tv2;
      wV0 = wV1;
      wV1 = wV2;
      xv0 = xv1;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        Bm0[q] = Bm1[q];
        Bm1[q] = Bm2[q];
      }
#pragma unroll
      for (int t = 0; t < JT; ++t) jv0[t] = jv1[t];
    }
  }
  // the virtual waves' sums added in virtual-wave order (wave, then group)
  sfa[wave][lane] = facc;
  __syncthreads();
  const int E = R * R + R;
  for (int w = 0; w < W; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < BT; ++t) {
        const int b = lane + 64 * t;
        if (b < nbs * nbs) {
          const int r0 = BS * (b / nbs), s0 = BS * (b % nbs);
#pragma unroll
          for (int q = 0; q < BS * BS; ++q) {
            const int r = r0 + q / BS, c = s0 + q % BS;
            if (r < R && c < R) {
              double v = w == 0 ? 0.0 : red[r * R + c];
#pragma unroll
              for (int g = 0; g < G; ++g) v += kacc[g][t][q];
              red[r * R + c] = v;
            }
          }
        }
      }
      if (lane < R) {
        double v = w == 0 ? 0.0 : red[R * R + lane];
        for (int g = 0; g < G; ++g) v += sfa[w][g * LG + lane];
        red[R * R + lane] = v;
      }
    }
    __syncthreads();
  }
  double* out = I.part_cub + (size_t)bx * E;
  for (int p = threadIdx.x; p < E; p += 64 * W) stg<double>(out + p, red[p]);
}

template <typename T, int RB, int W>
__global__ __launch_bounds__(64 * W) void k_cubature(const Inst<T>* __restrict__ tab, int m) {
  cubature_block<T, RB, W>(tab, blockIdx.x, blockIdx.y, m);
}

// Launches of at least kCubPackBlocks blocks of tets (batched instances,
// large meshes) with R <= 16 take the packed form, one wave of four lane
// groups; smaller launches and larger R the 4-wave form.  Both give the same
// bits.
static const int kCubPackBlocks = 1024;

template <typename T>
void launch_cubature(const Inst<T>* tab, int nb, int max_cblk, int max_r, hipStream_t s) {
  const int m = cubature_merge(nb, max_cblk);
  const dim3 grid((max_cblk + m - 1) / m, nb);
  const bool pack = (long long)nb * max_cblk >= kCubPackBlocks;
  if (max_r <= 8) {
    if (pack) k_cubature<T, 8, 1><<<grid, 64, 0, s>>>(tab, m);
    else k_cubature<T, 8, 4><<<grid, 256, 0, s>>>(tab, m);
  } else if (max_r <= 16) {
    if (pack) k_cubature<T, 16, 1><<<grid, 64, 0, s>>>(tab, m);
    else k_cubature<T, 16, 4><<<grid, 256, 0, s>>>(tab, m);
  } else {
    // R > 16: a packed form needs two accumulator sets of 16 FP64 values per
    // lane (270 registers, one wave per SIMD) and measured slower
    k_cubature<T, NMR_MAX_R, 4><<<grid, 256, 0, s>>>(tab, m);
  }
}
template void launch_cubature<float>(const Inst<float>*, int, int, int, hipStream_t);
template void launch_cubature<double>(const Inst<double>*, int, int, int, hipStream_t);


template <typename T>
__global__ void k_fint(const Inst<T>* __restrict__ tab, T* f_int) {
  const Inst<T>& I = tab[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < I.N) f_int[i] = (T)fint_at(I, i);
}
template <typename T>
void launch_fint(const Inst<T>* tab, T* f_int, int N, hipStream_t s) {
  k_fint<T><<<(N + 255) / 256, 256, 0, s>>>(tab, f_int);
}
template void launch_fint<float>(const Inst<float>*, float*, int, hipStream_t);
template void launch_fint<double>(const Inst<double>*, double*, int, hipStream_t);


// ---------------------------------------------------------------------------
// Mass terms over 256-DOF chunks.  With Jt_i = [U_i, J_i], w_r = r - rbar -
// dt rdot_bar, v_i = m_i (Jt_i . w_r + Hdd_i) - dt^2 m_i g_c:
//   a_i      = v_i + dt^2 f_int_i          (so phi = Jt^T a, eq. our_eq.)
//   G_kl    += m_i Jt_ik Jt_il             (Jt^T M Jt)
//   E_kj    += m_i Jt_ik dJ_ij             (Jt^T M [0, dJ])
//   phim_k  += Jt_ik v_i                   (phi without dt^2 Jt^T f_int)
//   uta_k   += U_ik (P a)_i                (filter transpose of the seed)
// i.e. one product Jt^T Y with Y_i = [m_i Jt_i, m_i dJ_i, v_i, (P a)_i],
// computed on the FP64 matrix cores (v_mfma_f64_16x16x4: A = Jt^T over four
// DOFs, B = four rows of Y), one partial per block, the four wave partials
// added in wave order.
// ---------------------------------------------------------------------------
#define MASS_ROWS 256
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
__global__ __launch_bounds__(256) void k_mass(const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  if (!I.active) return;
  if ((int)blockIdx.x >= I.n_mblk) return;
  const int R = I.R, np = I.n_p, nq = I.n_q, Cf = I.Cf, N = I.N;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __shared__ double wr[NMR_MAX_R];
  __shared__ double sm[MASS_ROWS], sv[MASS_ROWS], ss[MASS_ROWS];
  __shared__ double tile[2 * 16][5 * 16];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sJ = reinterpret_cast<T*>(smem_raw);  // [MASS_ROWS][R]
  T* sdJ = sJ + MASS_ROWS * R;               // [MASS_ROWS][nq]
  const double dt = I.dt;
  const int i0 = blockIdx.x * MASS_ROWS;
  // one DOF per thread; every load is issued first, from indices clamped
  // into range, then w_r, then Jt_i and dJ_i are staged and v_i, a_i and the
  // seed formed
  const int t = threadIdx.x;
  const int i = i0 + t;
  const int ic = min(i, N - 1);
  const T* rr = I.rec + (size_t)ic * Cf;
  T jv[NMR_MAX_R], djv[NMR_MAX_R], uv[NMR_MAX_R];
#pragma unroll
  for (int j = 0; j < NMR_MAX_R; ++j) {
    jv[j] = ldg<T>(rr + 1 + min(j, nq - 1));
    djv[j] = ldg<T>(rr + 1 + nq + min(j, nq - 1));
  }
  if (np > 0) {
#pragma unroll
    for (int k = 0; k < NMR_MAX_R; ++k) uv[k] = ldg<T>(I.U + (size_t)ic * np + min(k, np - 1));
  }
  const T hdd = ldg<T>(rr + 1 + 2 * nq);
  const double m_i = (double)ldg<T>(I.mass + ic), keep_i = (double)ldg<T>(I.keep + ic);
  const int lr = min(t, R - 1);
  const double wrv = ldg<double>(I.r + lr) - ldg<double>(I.rbar + lr) - dt * ldg<double>(I.rdot + lr);
  // a coupled domain's tie force counts as internal force
  const double fi = fint_at(I, ic) + (I.pen ? (double)ldg<T>(I.pen + ic) : 0.0);
  if (t < R) wr[t] = wrv;
  __syncthreads();
  {
    double m = 0.0, v = 0.0, s = 0.0;
    if (i < N) {
      m = m_i;
      double jw = 0.0;
#pragma unroll
      for (int k = 0; k < NMR_MAX_R; ++k)
        if (k < np) {
          sJ[t * R + k] = uv[k];
          jw += (double)uv[k] * wr[k];
        }
#pragma unroll
      for (int j = 0; j < NMR_MAX_R; ++j)
        if (j < nq) {
          sJ[t * R + np + j] = jv[j];
          sdJ[t * nq + j] = djv[j];
          jw += (double)jv[j] * wr[np + j];
        }
      v = m * (jw + (double)hdd) - dt * dt * m * I.g[i % 3];
      const double a = v + dt * dt * fi;
      s = keep_i * a;
      stg<T>(I.seed + i, (T)s);
    } else {
      for (int k = 0; k < R; ++k) sJ[t * R + k] = T(0);
      for (int j = 0; j < nq; ++j) sdJ[t * nq + j] = T(0);
    }
    sm[t] = m;
    sv[t] = v;
    ss[t] = s;
  }
  __syncthreads();
  // Jt^T Y on the FP64 matrix cores: each wave takes 64 DOFs, 4 per MFMA
  const int nrb = (R + 15) / 16;
  const int ny = R + nq + 2;
  const int ncb = (ny + 15) / 16;
  const int col = lane & 15, kk = lane >> 4;
  f64x4 acc[2][5];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 5; ++cb) acc[rb][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
  auto jt = [&](int lrow, int c) -> double { return c < R ? (double)sJ[lrow * R + c] : 0.0; };
  for (int step = 0; step < 16; ++step) {
    const int lrow = wave * 64 + step * 4 + kk;
    double a[2], b[5];
    const double m = sm[lrow];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) a[rb] = (rb < nrb) ? jt(lrow, rb * 16 + col) : 0.0;
#pragma unroll
    for (int cb = 0; cb < 5; ++cb) {
      const int n = cb * 16 + col;
      double y = 0.0;
      if (cb < ncb) {
        if (n < R) y = m * jt(lrow, n);
        else if (n < R + nq) y = m * (double)sdJ[lrow * nq + (n - R)];
        else if (n == R + nq) y = sv[lrow];
        else if (n == R + nq + 1) y = ss[lrow];
      }
      b[cb] = y;
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 5; ++cb)
        if (rb < nrb && cb < ncb) acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
  }
  // wave partial tiles added in wave order; the f64 16x16x4 result layout is
  // row-interleaved: item q of lane l is D[4*q + l/16][l%16]
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 5; ++cb)
          if (rb < nrb && cb < ncb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int rr = rb * 16 + 4 * q + kk, cc = cb * 16 + col;
              tile[rr][cc] = (w == 0 ? 0.0 : tile[rr][cc]) + acc[rb][cb][q];
            }
    }
    __syncthreads();
  }
  const int E = R * R + R * nq + R + np;
  double* out = I.part_mass + (size_t)blockIdx.x * E;
  for (int e = threadIdx.x; e < E; e += 256) {
    double v;
    if (e < R * R) v = tile[e / R][e % R];
    else if (e < R * R + R * nq) {
      const int e2 = e - R * R;
      v = tile[e2 / nq][R + e2 % nq];
    } else if (e < R * R + R * nq + R) v = tile[e - R * R - R * nq][R + nq];
    else v = tile[e - R * R - R * nq - R][R + nq + 1];
    stg<double>(out + e, v);
  }
}

template <typename T>
void launch_mass(const Inst<T>* tab, int nb, int max_mblk, int R, int nq, hipStream_t s) {
  const size_t lds = (size_t)MASS_ROWS * (R + nq) * sizeof(T);
  k_mass<T><<<dim3(max_mblk, nb), 256, lds, s>>>(tab);
}
template void launch_mass<float>(const Inst<float>*, int, int, int, int, hipStream_t);
template void launch_mass<double>(const Inst<double>*, int, int, int, int, hipStream_t);

// seed = P a for a caller vector a, with the U^T P a partials (other
// entries of the mass partials are zeroed) -- decoder_jacobian_hessian path.
template <typename T>
__global__ __launch_bounds__(256) void k_seed_from_a(const Inst<T>* __restrict__ tab, const T* a) {
  const Inst<T>& I = tab[blockIdx.y];
  if (!I.active) return;
  if ((int)blockIdx.x >= I.n_mblk) return;
  const int R = I.R, np = I.n_p, nq = I.n_q;
  __shared__ double ss[MASS_ROWS];
  const int t = threadIdx.x;
  const int i = blockIdx.x * MASS_ROWS + t;
  double s = 0.0;
  if (i < I.N) {
    s = (double)I.keep[i] * (double)a[i];
    I.seed[i] = (T)s;
  }
  ss[t] = s;
  __syncthreads();
  const int E = R * R + R * nq + R + np;
  double* out = I.part_mass + (size_t)blockIdx.x * E;
  for (int e = threadIdx.x; e < E; e += 256) {
    double acc = 0.0;
    const int k = e - (R * R + R * nq + R);
    if (k >= 0) {
      for (int q = 0; q < MASS_ROWS; ++q) {
        const int ii = blockIdx.x * MASS_ROWS + q;
        if (ii < I.N) acc += (double)I.U[(size_t)ii * np + k] * ss[q];
      }
    }
    out[e] = acc;
  }
}

template <typename T>
void launch_seed_from_a(const Inst<T>* tab, const T* a, int nb, int max_mblk, hipStream_t s) {
  k_seed_from_a<T><<<dim3(max_mblk, nb), 256, 0, s>>>(tab, a);
}
template void launch_seed_from_a<float>(const Inst<float>*, const float*, int, int, hipStream_t);
template void launch_seed_from_a<double>(const Inst<double>*, const double*, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Gram path of the mass terms (n_p = 0).  The output layer is linear and the
// lumped mass constant, so with the folded last-hidden activations F (columns
// F_J = J e_j, F_dJ, F_Hdd before W_L), y = F_J w_r + F_Hdd,
// Gam = W_L^T diag(m keep) W_L and gam = W_L^T (keep c), c_i = -dt^2 m_i g_c:
//   Jt^T M Jt = F_J^T Gam F_J,  Jt^T M dJ = F_J^T Gam F_dJ,
//   phim = F_J^T (Gam y + gam),  and the backprop seed W_L^T P a equals
//   Gam y + gam + dt^2 W_L^T P f_int  (the last term over cubature DOFs only).
// Each block takes 16 rows of Gam: T = Gam[rows] X with X = [F_J, F_dJ, y] on
// the FP64 matrix cores (4 waves split K), then one mass partial
// F_J[rows]^T T and its 16 entries of Gam y + gam as a backprop partial.
// ---------------------------------------------------------------------------
template <typename T, int NCB>
__device__ __forceinline__ void gram_block(const Inst<T>* __restrict__ tab, int bx, int by, int K) {
  const Inst<T>& I = tab[by];
  load_now(I.active, I.gram, I.n_gblk, I.n_q, I.R, I.fold, I.dt, I.Gam, I.gam, I.r, I.rbar, I.rdot, I.part_bwd,
           I.n_sblk, I.part_mass);
  if (!I.active) return;
  if (!I.gram || bx >= I.n_gblk) return;
  const int nq = I.n_q, R = I.R;  // R = n_q on this path
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, kk = lane >> 4;
  // rows [row0, row0 + 16) over the K part [kb0, kb0 + kh): each part has
  // its own partials (the mass terms and T y are linear in the K sum), gam
  // is added by part 0
  const int rb = bx / kGramKParts, kpart = bx - rb * kGramKParts;
  const int row0 = rb * 16, kh = K / kGramKParts, kb0 = kpart * kh;
  const T* F = I.fold;  // [Cf][K], K <= 256
  __shared__ double wr[NMR_MAX_R];
  __shared__ double y[256];
  __shared__ double tile[16][4 * 16];
  __shared__ double frow[NMR_MAX_R][16];  // F_J[row0 .. row0 + 15], column-major by j
  const double dt = I.dt;
  // X columns: F_J, F_dJ, y in NCB = ceil((2 n_q + 1) / 16) column blocks
  // Every global load is issued before the first wait, from indices clamped
  // into range: the folded columns of y (thread k), this wave's K-steps of
  // Gam and of X, the 16 F_J rows of the mass partial and the state.
  // NCB column blocks hold 2 n_q + 1 < 16 NCB columns, so n_q < QM
  constexpr int QM = 8 * NCB;
  static_assert(QM <= NMR_MAX_R, "column blocks");
  const int kt = kb0 + min((int)threadIdx.x, kh - 1);
  T fy[QM];
#pragma unroll
  for (int j = 0; j < QM; ++j) fy[j] = ldg<T>(F + (size_t)(1 + min(j, nq - 1)) * K + kt);
  const T fh = ldg<T>(F + (size_t)(1 + 2 * nq) * K + kt);
  constexpr int NST = 256 / (16 * kGramKParts);  // K-steps of one wave at K = 256 (kh/4 entries, 4 per step)
  const int kper = kh / 4, nst = kper / 4;
  const double* G = I.Gam + (size_t)(row0 + col) * K;
  double av[NST];
  T bv[NST][NCB];
#pragma unroll
  for (int st = 0; st < NST; ++st) {
    const int k = kb0 + min(wave * kper + 4 * st + kk, kh - 1);
    av[st] = ldg<double>(G + k);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) bv[st][cb] = ldg<T>(F + (size_t)(1 + min(cb * 16 + col, 2 * nq - 1)) * K + k);
  }
  constexpr int FP = (QM * 16 + 255) / 256;
  T fpv[FP];
#pragma unroll
  for (int q = 0; q < FP; ++q) {
    const int p = threadIdx.x + 256 * q;
    fpv[q] = ldg<T>(F + (size_t)(1 + min(p >> 4, nq - 1)) * K + row0 + (p & 15));
  }
  const double gm = ldg<double>(I.gam + row0 + (threadIdx.x & 15));
  const int lr = min((int)threadIdx.x, R - 1);
  const double wrv = ldg<double>(I.r + lr) - ldg<double>(I.rbar + lr) - dt * ldg<double>(I.rdot + lr);
  if ((int)threadIdx.x < R) wr[threadIdx.x] = wrv;
#pragma unroll
  for (int q = 0; q < FP; ++q) {
    const int p = threadIdx.x + 256 * q;
    if ((p >> 4) < nq) frow[p >> 4][p & 15] = (double)fpv[q];
  }
  __syncthreads();
  if ((int)threadIdx.x < kh) {
    double v = (double)fh;
#pragma unroll
    for (int j = 0; j < QM; ++j)
      if (j < nq) v += (double)fy[j] * wr[j];
    y[threadIdx.x] = v;
  }
  __syncthreads();
  f64x4 acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = f64x4{0.0, 0.0, 0.0, 0.0};
  // each wave a quarter of the block's K part, 4 entries per step, in
  // increasing k.  The y entries of the wave's steps are read from LDS in one
  // batch and every B operand is chosen by selects; steps past the quarter
  // (K < 256) multiply a zero A operand, which adds exact zeros, so the loop
  // is straight-line code
  double yv[NST];
#pragma unroll
  for (int st = 0; st < NST; ++st) yv[st] = y[min(wave * kper + 4 * st + kk, kh - 1)];
#pragma unroll
  for (int st = 0; st < NST; ++st) {
    const double a = st < nst ? av[st] : 0.0;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int n = cb * 16 + col;
      const double fb = n < 2 * nq ? (double)bv[st][cb] : 0.0;
      const double b = n == 2 * nq ? yv[st] : fb;
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb], 0, 0, 0);
    }
  }
  // wave partial tiles added in wave order (f64 result rows interleaved)
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = 4 * q + kk, cc = cb * 16 + col;
          tile[rr][cc] = (w == 0 ? 0.0 : tile[rr][cc]) + acc[cb][q];
        }
    }
    __syncthreads();
  }
  // T_y + gam for these rows: the backprop partial after the sparse blocks
  if (threadIdx.x < 16) {
    const double zb = tile[threadIdx.x][2 * nq] + (kpart == 0 ? gm : 0.0);
    tile[threadIdx.x][2 * nq] = zb;
    stg<double>(I.part_bwd + (size_t)(I.n_sblk + kpart) * K + row0 + threadIdx.x, zb);
  }
  __syncthreads();
  // mass partial F_J[rows]^T T in the layout of the direct path
  const int E = R * R + R * nq + R;
  double* out = I.part_mass + (size_t)bx * E;
  for (int e = threadIdx.x; e < E; e += 256) {
    int i, c;
    if (e < R * R) {
      i = e / R;
      c = e % R;
    } else if (e < R * R + R * nq) {
      i = (e - R * R) / nq;
      c = nq + (e - R * R) % nq;
    } else {
      i = e - R * R - R * nq;
      c = 2 * nq;
    }
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) v += frow[i][r] * tile[r][c];
    stg<double>(out + e, v);
  }
}

template <typename T, int NCB>
__global__ __launch_bounds__(256) void k_gram(const Inst<T>* __restrict__ tab, int K) {
  gram_block<T, NCB>(tab, blockIdx.x, blockIdx.y, K);
}

// The cubature pass and the Gram kernel in one launch (the Gram terms need
// only the folded activations and the state, not the decoded rows): blocks
// below n_cub_blocks run the cubature, the rest the Gram rows.
template <typename T, int NCB, int RB>
__global__ __launch_bounds__(256) void k_cub_gram(const Inst<T>* __restrict__ tab, int m, int K, int n_cub_blocks) {
  if ((int)blockIdx.x < n_cub_blocks) cubature_block<T, RB, 4>(tab, blockIdx.x, blockIdx.y, m);
  else gram_block<T, NCB>(tab, blockIdx.x - n_cub_blocks, blockIdx.y, K);
}

template <typename T>
void launch_gram(const Inst<T>* tab, int nb, int max_gblk, int K, int nq, hipStream_t s) {
  const dim3 grid(max_gblk, nb);
  switch ((2 * nq + 1 + 15) / 16) {
    case 1: k_gram<T, 1><<<grid, 256, 0, s>>>(tab, K); break;
    case 2: k_gram<T, 2><<<grid, 256, 0, s>>>(tab, K); break;
    case 3: k_gram<T, 3><<<grid, 256, 0, s>>>(tab, K); break;
    default: k_gram<T, 4><<<grid, 256, 0, s>>>(tab, K); break;
  }
}
template void launch_gram<float>(const Inst<float>*, int, int, int, int, hipStream_t);
template void launch_gram<double>(const Inst<double>*, int, int, int, int, hipStream_t);

template <typename T, int RB>
static void cub_gram_ncb(const Inst<T>* tab, int nb, int m, int ncb, int max_gblk, int K, int nq, hipStream_t s) {
  const dim3 grid(ncb + max_gblk, nb);
  switch ((2 * nq + 1 + 15) / 16) {
    case 1: k_cub_gram<T, 1, RB><<<grid, 256, 0, s>>>(tab, m, K, ncb); break;
    case 2: k_cub_gram<T, 2, RB><<<grid, 256, 0, s>>>(tab, m, K, ncb); break;
    case 3: k_cub_gram<T, 3, RB><<<grid, 256, 0, s>>>(tab, m, K, ncb); break;
    default: k_cub_gram<T, 4, RB><<<grid, 256, 0, s>>>(tab, m, K, ncb); break;
  }
}

template <typename T>
void launch_cub_gram(const Inst<T>* tab, int nb, int max_cblk, int max_gblk, int K, int nq, hipStream_t s) {
  const int m = cubature_merge(nb, max_cblk), ncb = (max_cblk + m - 1) / m;
  // the Gram path has no linear subspace: R = n_q
  if (nq <= 8) cub_gram_ncb<T, 8>(tab, nb, m, ncb, max_gblk, K, nq, s);
  else if (nq <= 16) cub_gram_ncb<T, 16>(tab, nb, m, ncb, max_gblk, K, nq, s);
  else cub_gram_ncb<T, NMR_MAX_R>(tab, nb, m, ncb, max_gblk, K, nq, s);
}
template void launch_cub_gram<float>(const Inst<float>*, int, int, int, int, int, hipStream_t);
template void launch_cub_gram<double>(const Inst<double>*, int, int, int, int, int, hipStream_t);

// setup: Gam = W_L^T diag(m keep) W_L over the N rows of this instance and
// gam = W_L^T (keep c); one thread per entry, rows in order
template <typename TW>
__device__ inline double wload(const TW* p) { return (double)(float)*p; }
template <>
__device__ inline double wload<double>(const double* p) { return *p; }

template <typename T, typename TW>
__global__ __launch_bounds__(256) void k_gram_setup(const TW* __restrict__ W, int K, const T* mass, const T* keep,
                                                    int N, double dt, double g0, double g1, double g2, double* Gam,
                                                    double* gam) {
  const int k = blockIdx.x * 16 + (threadIdx.x & 15);
  const int l = blockIdx.y * 16 + (threadIdx.x >> 4);
  double acc = 0.0;
  if (blockIdx.y < (unsigned)(K / 16)) {
    for (int i = 0; i < N; ++i)
      acc += wload(W + (size_t)i * K + k) * wload(W + (size_t)i * K + l) * (double)mass[i] * (double)keep[i];
    Gam[(size_t)k * K + l] = acc;
  } else if (threadIdx.x < 16) {
    const double g[3] = {g0, g1, g2};
    for (int i = 0; i < N; ++i)
      acc += wload(W + (size_t)i * K + k) * (double)keep[i] * (-dt * dt * (double)mass[i] * g[i % 3]);
    gam[k] = acc;
  }
}

template <typename T>
void launch_gram_setup(const void* W, int prec, int K, const T* mass, const T* keep, int N, double dt,
                       const double* g, double* Gam, double* gam, hipStream_t s) {
  dim3 grid(K / 16, K / 16 + 1);
  if (prec == PREC_BF16)
    k_gram_setup<T, __bf16><<<grid, 256, 0, s>>>((const __bf16*)W, K, mass, keep, N, dt, g[0], g[1], g[2], Gam, gam);
  else if (prec == PREC_FP64)
    k_gram_setup<T, double><<<grid, 256, 0, s>>>((const double*)W, K, mass, keep, N, dt, g[0], g[1], g[2], Gam, gam);
  else
    k_gram_setup<T, float><<<grid, 256, 0, s>>>((const float*)W, K, mass, keep, N, dt, g[0], g[1], g[2], Gam, gam);
}
template void launch_gram_setup<float>(const void*, int, int, const float*, const float*, int, double, const double*,
                                       double*, double*, hipStream_t);
template void launch_gram_setup<double>(const void*, int, int, const double*, const double*, int, double,
                                        const double*, double*, double*, hipStream_t);


// ---------------------------------------------------------------------------
// Fixed-order sums of the cubature and mass partials (sums_block).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_sums(const Inst<T>* __restrict__ tab, int cub_m) {
  sums_block<T>(tab, blockIdx.x, blockIdx.y, cub_m);
}

template <typename T>
void launch_sums(const Inst<T>* tab, int nb, int max_entries, int max_cblk, hipStream_t s) {
  k_sums<T><<<dim3((max_entries + 15) / 16, nb), 256, 0, s>>>(tab, cubature_merge(nb, max_cblk));
}
template void launch_sums<float>(const Inst<float>*, int, int, int, hipStream_t);
template void launch_sums<double>(const Inst<double>*, int, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Assemble A = Jt^T M [U, J + dJ] + dt^2 Kr + diag(0, a . H) and
// phi = phim + dt^2 fr (eq. system_mat with the sign differentiation gives),
// record ||phi||, solve A delta = -phi and update r += delta.  On the last
// iteration of a step: rdot = (r - rbar)/dt, rbar = r.  A failed instance
// keeps its last good (rbar, rdot).
//
// The solve is Gauss-Jordan elimination with partial pivoting on the
// augmented matrix [A | -phi], held in registers across one wavefront: lane
// (g, c) = (lane / CW, lane % CW) owns column c (c == R is the right-hand
// side) of rows g, g + G, g + 2G, ...  (G = 64 / CW).  Rows are not moved;
// the pivot of column k is the row of largest |a_ik| among the rows not yet
// pivots, compared on the top bits of |a_ik| (sign, exponent and 14 mantissa
// bits) with ties to the lower row, so a chosen pivot is within a factor
// 1 + 2^-14 of the largest.  The pivot row is divided by its pivot and
// eliminated from every other row; after R steps the right-hand column of
// pivot row p_k holds delta_k.  Every value is broadcast through the LDS
// crossbar (ds_bpermute) or readlane: no LDS round trip or barrier per step.
// ---------------------------------------------------------------------------
__device__ inline double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
__device__ inline double bperm_f64(double v, int src_lane) {
  const int addr = src_lane << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ inline unsigned abs_hi(double v) { return (unsigned)__double2hiint(v) & 0x7FFFFFFFu; }

template <typename T, int CW>
__device__ inline void solve_body(const Inst<T>& I, int iter, int mode, double* A_out, double* phi_out) {
  constexpr int G = 64 / CW, RPL = CW / G;
  const int R = I.R, np = I.n_p, nq = I.n_q, lane = threadIdx.x;
  const int g = lane / CW, c = lane % CW;
  const double dt = I.dt, dt2 = dt * dt;
  const auto* Gm = gp(I.sum_mass);
  const auto* E = Gm + R * R;
  const auto* phim = E + R * nq;
  const auto* Kr = gp(I.sum_cub);
  const auto* fr = Kr + R * R;
  // Bq is n_q x n_q; with n_q = 0 any valid address stands in (never used)
  const auto* Bq = nq > 0 ? gp(I.Bq) : Gm;
  const bool row = lane < R;
  // every global load of the kernel is issued here, unconditionally and from
  // indices clamped into range, so that they are all in flight together
  const int st0 = *gp(I.status);
  const int lr = min(lane, R - 1);
  const double r_l = row ? gp(I.r)[lr] : 0.0;
  const double rbar_l = row ? gp(I.rbar)[lr] : 0.0;
  const double rdot_l = row ? gp(I.rdot)[lr] : 0.0;
  const int cc = min(c, R - 1), cq = max(cc - np, 0);
  double a[RPL];
#pragma unroll
  for (int m = 0; m < RPL; ++m) {
    const int i = g + G * m;
    const int ii = min(i, R - 1), iq = max(ii - np, 0);
    const double gk = Gm[ii * R + cc] + dt2 * Kr[ii * R + cc];
    const double e = E[ii * nq + cq];
    const double bq = Bq[nq > 0 ? iq * nq + cq : 0];
    const double ph = phim[ii] + dt2 * fr[ii];
    double v = gk;
    if (c >= np) v += e;
    if (ii >= np && c >= np) v += bq;
    a[m] = i >= R ? 0.0 : c < R ? v : c == R ? -ph : 0.0;
  }
  bool fin = true;
  unsigned hmax = 0;
  double ss = 0.0;
#pragma unroll
  for (int m = 0; m < RPL; ++m) {
    fin = fin && isfinite(a[m]);
    if (c < R) hmax = max(hmax, abs_hi(a[m]));
    ss = fma(a[m], a[m], ss);  // nonzero only in the right-hand column
  }
  double nrm2 = 0.0;
#pragma unroll
  for (int gg = 0; gg < G; ++gg) nrm2 += readlane_f64(ss, gg * CW + R);
  for (int off = 32; off > 0; off >>= 1) hmax = max(hmax, (unsigned)__shfl_xor((int)hmax, off));
  const double amax = __hiloint2double((int)hmax, 0);
  const bool all_finite = __all(fin);
  int st = st0;
  if (!all_finite && st == 0) st = ST_NONFINITE;
  if (lane == 0) {
    gpw(I.resid)[iter] = sqrt(nrm2);
    if (st != st0) atomicOr(I.status, st);
  }
  if (mode & SOLVE_WRITE_SYSTEM) {
#pragma unroll
    for (int m = 0; m < RPL; ++m) {
      const int i = g + G * m;
      if (i < R) {
        if (c < R) gpw(A_out)[i * R + c] = a[m];
        else if (c == R) gpw(phi_out)[i] = -a[m];
      }
    }
  }
  if (!(mode & SOLVE_UPDATE) || st != 0) return;

  __shared__ int piv[NMR_MAX_R];
  __shared__ double xcol[NMR_MAX_R];
  unsigned used = 0;  // bit i: row i has been a pivot (uniform)
  bool singular = false;
  for (int k = 0; k < R; ++k) {
    // column k of this lane's rows (independent of the pivot: issued first)
    double f[RPL];
#pragma unroll
    for (int m = 0; m < RPL; ++m) f[m] = bperm_f64(a[m], g * CW + k);
    unsigned key = 0;
#pragma unroll
    for (int m = 0; m < RPL; ++m) {
      const int i = g + G * m;
      const unsigned kv = (abs_hi(a[m]) & ~63u) | (unsigned)(63 - i);
      key = (i < R && !((used >> i) & 1u)) ? max(key, kv) : key;
    }
    unsigned best = 0;
#pragma unroll
    for (int gg = 0; gg < G; ++gg) best = max(best, (unsigned)__builtin_amdgcn_readlane((int)key, gg * CW + k));
    const int p = 63 - (int)(best & 63u);  // best >= 32: some row < R is unused
    const int mp = p / G, src = (p % G) * CW;
    double sel = a[0];
#pragma unroll
    for (int m = 1; m < RPL; ++m) sel = (m == mp) ? a[m] : sel;
    const double apk = readlane_f64(sel, src + k);
    if (!(fabs(apk) > 1e-300 * amax)) {
      singular = true;
      break;
    }
    const double prn = bperm_f64(sel, src + c) / apk;  // pivot row, divided by its pivot
#pragma unroll
    for (int m = 0; m < RPL; ++m) a[m] = (g + G * m == p) ? prn : fma(-f[m], prn, a[m]);
    used |= 1u << p;
    if (lane == 0) piv[k] = p;
  }
  if (singular) {
    if (lane == 0) atomicOr(I.status, ST_SINGULAR);
    return;
  }
  if (c == R) {
#pragma unroll
    for (int m = 0; m < RPL; ++m)
      if (g + G * m < R) xcol[g + G * m] = a[m];
  }
  __syncthreads();
  // new state from registers; the decoder input of the next iteration is
  // taken from the lanes of the q block (exchange through LDS)
  const double rn = r_l + (row ? xcol[piv[lane]] : 0.0);
  const bool fin_step = mode & SOLVE_FINISH;
  const double rbar_n = fin_step ? rn : rbar_l;
  const double rdot_n = fin_step ? (rn - rbar_l) / dt : rdot_l;
  __shared__ double sq[3][NMR_MAX_R];
  if (row) {
    gpw(I.r)[lane] = rn;
    if (fin_step) {
      gpw(I.rdot)[lane] = rdot_n;
      gpw(I.rbar)[lane] = rbar_n;
    }
    if (lane >= np) {
      sq[0][lane - np] = rn;
      sq[1][lane - np] = rn - rbar_n;
      sq[2][lane - np] = rdot_n;
    }
  }
  __syncthreads();
  if (lane < nq) {
    auto* din = gpw(I.dec_in);
    din[lane] = sq[0][lane];
    din[nq + lane] = sq[1][lane];
    din[2 * nq + lane] = sq[2][lane];
  }
}

template <typename T>
__global__ __launch_bounds__(64) void k_solve(const Inst<T>* __restrict__ tab, int iter, int mode, double* A_out,
                                              double* phi_out) {
  const Inst<T>& I = tab[blockIdx.y];
  load_now(I.active, I.R, I.n_p, I.n_q, I.dt, I.sum_mass, I.sum_cub, I.Bq, I.status, I.r, I.rbar, I.rdot, I.resid,
           I.dec_in);
  if (!I.active) return;
  if (mode & SOLVE_WRITE_INST) {
    A_out = I.sysA;
    phi_out = I.sysphi;
  }
  if (I.R < 16) solve_body<T, 16>(I, iter, mode, A_out, phi_out);
  else solve_body<T, 32>(I, iter, mode, A_out, phi_out);
}

template <typename T>
void launch_solve(const Inst<T>* tab, int nb, int iter, int mode, double* A_out, double* phi_out, hipStream_t s) {
  k_solve<T><<<dim3(1, nb), 64, 0, s>>>(tab, iter, mode, A_out, phi_out);
}
template void launch_solve<float>(const Inst<float>*, int, int, int, double*, double*, hipStream_t);
template void launch_solve<double>(const Inst<double>*, int, int, int, double*, double*, hipStream_t);

}  // namespace nmr
