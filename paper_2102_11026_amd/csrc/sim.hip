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
// ---------------------------------------------------------------------------
__device__ inline double softplus(double x) { return x > 0.0 ? x + log1p(exp(-x)) : log1p(exp(x)); }

template <typename T>
__global__ __launch_bounds__(256) void k_step_begin(const Inst<T>* __restrict__ tab, int mode) {
  const Inst<T>& I = tab[blockIdx.y];
  const int R = I.R, np = I.n_p, nq = I.n_q;
  if (mode == BEGIN_STEP)
    for (int k = threadIdx.x; k < R; k += 256) I.r[k] = I.rbar[k];
  if (I.wn_L > 0) {
    T* buf0 = I.wn_buf;
    T* buf1 = I.wn_buf + I.wn_maxw;
    const int W0 = I.wn_w[0];
    for (int k = threadIdx.x; k < W0; k += 256) buf0[k] = (T)I.rbar[k];
    __syncthreads();
    for (int l = 0; l < I.wn_L; ++l) {
      const T* in = (l & 1) ? buf1 : buf0;
      T* out = (l & 1) ? buf0 : buf1;
      const int wi = I.wn_w[l], wo = I.wn_w[l + 1];
      const bool last = (l == I.wn_L - 1);
      for (int o = threadIdx.x; o < wo; o += 256) {
        double acc = (double)I.wn_b[l][o];
        const T* Wr = I.wn_W[l] + (size_t)o * wi;
        for (int k = 0; k < wi; ++k) acc += (double)Wr[k] * (double)in[k];
        const double z = softplus(acc);
        if (last) I.cub_w[o] = (T)(I.wn_scale * z);
        else out[o] = (T)z;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nq; k += 256) {
    const double q = I.r[np + k];
    I.dec_in[k] = q;
    I.dec_in[nq + k] = q - I.rbar[np + k];
    I.dec_in[2 * nq + k] = I.rdot[np + k];
  }
}

template <typename T>
void launch_step_begin(const Inst<T>* tab, int nb, int mode, hipStream_t s) {
  k_step_begin<T><<<dim3(1, nb), 256, 0, s>>>(tab, mode);
}
template void launch_step_begin<float>(const Inst<float>*, int, int, hipStream_t);
template void launch_step_begin<double>(const Inst<double>*, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Cubature: one wave handles cub_per_blk tets.  Per tet e with deformation
// gradient F = D_s B_m, first Piola stress P and its tangent dP:
//   dF_r = dF/dr_r = sum_a Jt_{a,r} (x) g_a,   g_a = gradient of hat fn a,
//   fr_r += w V P : dF_r,   Kr_rs += w V dP[dF_r] : dF_s,
//   f_a   = w V P g_a (element force, scattered later by gather),
// which equals Jt_e^T f_e and Jt_e^T K_e Jt_e without forming the 12 x 12
// K_e.  Neo-Hookean: P = mu (F - F^-T) + lam ln J F^-T,
//   dP[dF] = mu dF + (mu - lam ln J) F^-T dF^T F^-T + lam tr(F^-1 dF) F^-T.
// Element math in T, accumulation in FP64.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_cubature(const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  if ((int)blockIdx.x >= I.n_cblk) return;
  const int R = I.R, lane = threadIdx.x;
  const int na = I.cu_na;
  const T mu = (T)I.mu, lam = (T)I.lam;
  __shared__ T xs[12];
  __shared__ T J12[12][NMR_MAX_R + 1];
  __shared__ T dFs[NMR_MAX_R][9];
  __shared__ T dPs[NMR_MAX_R][9];
  constexpr int KT = (NMR_MAX_R * NMR_MAX_R + 63) / 64;
  double kacc[KT];
#pragma unroll
  for (int i = 0; i < KT; ++i) kacc[i] = 0.0;
  double facc = 0.0;
  const int e0 = blockIdx.x * I.cub_per_blk;
  const int e1 = min(e0 + I.cub_per_blk, I.n_cub);
  for (int e = e0; e < e1; ++e) {
    const int* tv = I.cub_v + 4 * e;
    if (lane < 12) {
      const int dof = 3 * tv[lane / 3] + lane % 3;
      xs[lane] = I.X[dof] + I.cu_u[(size_t)dof * I.cu_u_ld];
    }
    for (int p = lane; p < 12 * R; p += 64) {
      const int ac = p / R, r = p - ac * R;
      const int dof = 3 * tv[ac / 3] + ac % 3;
      J12[ac][r] = (r < na) ? I.cu_Ja[(size_t)dof * I.cu_Ja_ld + r] : I.cu_Jb[(size_t)dof * I.cu_Jb_ld + (r - na)];
    }
    __syncthreads();
    // every lane: F, its inverse, P (uniform work, no divergence)
    const T* Bm = I.cub_Bm + 9 * e;
    T G[4][3];
    for (int j = 0; j < 3; ++j) {
      G[1][j] = Bm[0 * 3 + j];
      G[2][j] = Bm[1 * 3 + j];
      G[3][j] = Bm[2 * 3 + j];
      G[0][j] = -(G[1][j] + G[2][j] + G[3][j]);
    }
    T F[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T acc = T(0);
        for (int a = 1; a < 4; ++a) acc += (xs[3 * a + i] - xs[i]) * G[a][j];
        F[i][j] = acc;
      }
    const T det = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                  F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
    if (det <= T(0) && lane == 0) atomicOr(I.status, ST_INVERTED);
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
    const T wV = I.cu_w[e] * I.cub_Ve[e];
    const T c2 = mu - lam * lnJ;
    if (lane < R) {
      const int r = lane;
      T dF[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          T acc = T(0);
          for (int a = 0; a < 4; ++a) acc += J12[3 * a + i][r] * G[a][j];
          dF[i][j] = acc;
        }
      // tr(F^-1 dF) = A : dF
      T tr = T(0);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) tr += A[i][j] * dF[i][j];
      // M = dF^T A, then A M = A dF^T A
      T M[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = dF[0][i] * A[0][j] + dF[1][i] * A[1][j] + dF[2][i] * A[2][j];
      T fr = T(0);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          const T ADA = A[i][0] * M[0][j] + A[i][1] * M[1][j] + A[i][2] * M[2][j];
          dPs[r][3 * i + j] = mu * dF[i][j] + c2 * ADA + lam * tr * A[i][j];
          dFs[r][3 * i + j] = dF[i][j];
          fr += P[i][j] * dF[i][j];
        }
      facc += (double)wV * (double)fr;
    }
    if (lane < 12) {
      const int a = lane / 3, i = lane % 3;
      T f = T(0);
      for (int j = 0; j < 3; ++j) f += P[i][j] * G[a][j];
      I.fe[(size_t)e * 12 + lane] = wV * f;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const int p = lane + 64 * t;
      if (p < R * R) {
        const int r = p / R, s = p - r * R;
        T acc = T(0);
        for (int k = 0; k < 9; ++k) acc += dPs[r][k] * dFs[s][k];
        kacc[t] += (double)wV * (double)acc;
      }
    }
    __syncthreads();
  }
  const int E = R * R + R;
  double* out = I.part_cub + (size_t)blockIdx.x * E;
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int p = lane + 64 * t;
    if (p < R * R) out[p] = kacc[t];
  }
  if (lane < R) out[R * R + lane] = facc;
}

template <typename T>
void launch_cubature(const Inst<T>* tab, int nb, int max_cblk, hipStream_t s) {
  k_cubature<T><<<dim3(max_cblk, nb), 64, 0, s>>>(tab);
}
template void launch_cubature<float>(const Inst<float>*, int, int, hipStream_t);
template void launch_cubature<double>(const Inst<double>*, int, int, hipStream_t);

// f_int[i] = sum of the weighted element forces at DOF i (fixed CSR order)
template <typename T>
__device__ inline double fint_at(const Inst<T>& I, int i) {
  const int v = i / 3, c = i - 3 * v;
  double f = 0.0;
  for (int p = I.csr_ptr[v]; p < I.csr_ptr[v + 1]; ++p) {
    const int ent = I.csr_ent[p];
    f += (double)I.fe[(size_t)(ent >> 2) * 12 + 3 * (ent & 3) + c];
  }
  return f;
}

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
// and the backpropagation seed P a.  FP64 accumulation, one partial per
// block.
// ---------------------------------------------------------------------------
#define MASS_ROWS 256
template <typename T>
__global__ __launch_bounds__(256) void k_mass(const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  if ((int)blockIdx.x >= I.n_mblk) return;
  const int R = I.R, np = I.n_p, nq = I.n_q, Cf = I.Cf;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);      // [MASS_ROWS]
  double* sv = sm + MASS_ROWS;                            // [MASS_ROWS]
  double* ss = sv + MASS_ROWS;                            // [MASS_ROWS]
  __shared__ double wr[NMR_MAX_R];
  T* sJ = reinterpret_cast<T*>(ss + MASS_ROWS);           // [MASS_ROWS][R]
  T* sdJ = sJ + MASS_ROWS * R;                            // [MASS_ROWS][nq]
  const double dt = I.dt;
  if (threadIdx.x < R) wr[threadIdx.x] = I.r[threadIdx.x] - I.rbar[threadIdx.x] - dt * I.rdot[threadIdx.x];
  __syncthreads();
  const int t = threadIdx.x;
  const int i = blockIdx.x * MASS_ROWS + t;
  if (i < I.N) {
    const T* rr = I.rec + (size_t)i * Cf;
    const double m = (double)I.mass[i];
    double jw = 0.0;
    for (int k = 0; k < np; ++k) {
      const T u = I.U[(size_t)i * np + k];
      sJ[t * R + k] = u;
      jw += (double)u * wr[k];
    }
    for (int j = 0; j < nq; ++j) {
      const T Jv = rr[1 + j];
      sJ[t * R + np + j] = Jv;
      sdJ[t * nq + j] = rr[1 + nq + j];
      jw += (double)Jv * wr[np + j];
    }
    const double v = m * (jw + (double)rr[1 + 2 * nq]) - dt * dt * m * I.g[i % 3];
    const double a = v + dt * dt * fint_at(I, i);
    const double s = (double)I.keep[i] * a;
    I.seed[i] = (T)s;
    sm[t] = m;
    sv[t] = v;
    ss[t] = s;
  } else {
    for (int k = 0; k < R; ++k) sJ[t * R + k] = T(0);
    for (int j = 0; j < nq; ++j) sdJ[t * nq + j] = T(0);
    sm[t] = 0.0;
    sv[t] = 0.0;
    ss[t] = 0.0;
  }
  __syncthreads();
  const int E = R * R + R * nq + R + np;
  double* out = I.part_mass + (size_t)blockIdx.x * E;
  for (int e = threadIdx.x; e < E; e += 256) {
    double acc = 0.0;
    if (e < R * R) {
      const int k = e / R, l = e - k * R;
      for (int q = 0; q < MASS_ROWS; ++q) acc += sm[q] * (double)sJ[q * R + k] * (double)sJ[q * R + l];
    } else if (e < R * R + R * nq) {
      const int e2 = e - R * R;
      const int k = e2 / nq, j = e2 - k * nq;
      for (int q = 0; q < MASS_ROWS; ++q) acc += sm[q] * (double)sJ[q * R + k] * (double)sdJ[q * nq + j];
    } else if (e < R * R + R * nq + R) {
      const int k = e - R * R - R * nq;
      for (int q = 0; q < MASS_ROWS; ++q) acc += (double)sJ[q * R + k] * sv[q];
    } else {
      const int k = e - R * R - R * nq - R;
      for (int q = 0; q < MASS_ROWS; ++q) acc += (double)sJ[q * R + k] * ss[q];
    }
    out[e] = acc;
  }
}

template <typename T>
static size_t mass_lds(int R, int nq) {
  return 3 * MASS_ROWS * sizeof(double) + (size_t)MASS_ROWS * (R + nq) * sizeof(T);
}

template <typename T>
void launch_mass(const Inst<T>* tab, int nb, int max_mblk, int R, int nq, hipStream_t s) {
  k_mass<T><<<dim3(max_mblk, nb), 256, mass_lds<T>(R, nq), s>>>(tab);
}
template void launch_mass<float>(const Inst<float>*, int, int, int, int, hipStream_t);
template void launch_mass<double>(const Inst<double>*, int, int, int, int, hipStream_t);

// seed = P a for a caller vector a, with the U^T P a partials (other
// entries of the mass partials are zeroed) -- decoder_jacobian_hessian path.
template <typename T>
__global__ __launch_bounds__(256) void k_seed_from_a(const Inst<T>* __restrict__ tab, const T* a) {
  const Inst<T>& I = tab[blockIdx.y];
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
// Fixed-order sums of the cubature and mass partials.  Each block takes 64
// entries; four slices of 64 threads add every fourth block, then the four
// slice sums are added in order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_sums(const Inst<T>* __restrict__ tab) {
  const Inst<T>& I = tab[blockIdx.y];
  const int R = I.R;
  const int Ec = R * R + R;
  const int Em = R * R + R * I.n_q + R + I.n_p;
  const int kk = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + kk;
  __shared__ double part[4][64];
  double acc = 0.0;
  if (e < Ec) {
    for (int b = sl; b < I.n_cblk; b += 4) acc += I.part_cub[(size_t)b * Ec + e];
  } else if (e < Ec + Em) {
    const int e2 = e - Ec;
    for (int b = sl; b < I.n_mblk; b += 4) acc += I.part_mass[(size_t)b * Em + e2];
  }
  part[sl][kk] = acc;
  __syncthreads();
  if (sl == 0) {
    const double v = ((part[0][kk] + part[1][kk]) + part[2][kk]) + part[3][kk];
    if (e < Ec) I.sum_cub[e] = v;
    else if (e < Ec + Em) I.sum_mass[e - Ec] = v;
  }
}

template <typename T>
void launch_sums(const Inst<T>* tab, int nb, int max_entries, hipStream_t s) {
  k_sums<T><<<dim3((max_entries + 63) / 64, nb), 256, 0, s>>>(tab);
}
template void launch_sums<float>(const Inst<float>*, int, int, hipStream_t);
template void launch_sums<double>(const Inst<double>*, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Assemble A = Jt^T M [U, J + dJ] + dt^2 Kr + diag(0, a . H) and
// phi = phim + dt^2 fr (eq. system_mat with the sign differentiation gives),
// record ||phi||, LU with partial pivoting (one lane per row) and r += delta
// with A delta = -phi.  On the last iteration of a step: rdot = (r-rbar)/dt,
// rbar = r.  A failed instance keeps its last good (rbar, rdot).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_solve(const Inst<T>* __restrict__ tab, int iter, int mode, double* A_out,
                                              double* phi_out) {
  const Inst<T>& I = tab[blockIdx.y];
  const int R = I.R, np = I.n_p, nq = I.n_q, lane = threadIdx.x;
  const double dt = I.dt;
  __shared__ double A[NMR_MAX_R][NMR_MAX_R + 1];
  __shared__ double b[NMR_MAX_R];
  __shared__ double x[NMR_MAX_R];
  __shared__ int flag;
  __shared__ int st;
  const double* G = I.sum_mass;
  const double* E = G + R * R;
  const double* phim = E + R * nq;
  const double* Kr = I.sum_cub;
  const double* fr = Kr + R * R;
  for (int p = lane; p < R * R; p += 64) {
    const int k = p / R, l = p - k * R;
    double v = G[p] + dt * dt * Kr[p];
    if (l >= np) v += E[k * nq + (l - np)];
    if (k >= np && l >= np) v += I.Bq[(k - np) * nq + (l - np)];
    A[k][l] = v;
  }
  if (lane < R) b[lane] = phim[lane] + dt * dt * fr[lane];
  if (lane == 0) {
    flag = 0;
    st = __atomic_load_n(I.status, __ATOMIC_RELAXED);
  }
  __syncthreads();
  if (lane == 0) {
    double nrm = 0.0, amax = 0.0;
    bool finite = true;
    for (int k = 0; k < R; ++k) {
      nrm += b[k] * b[k];
      finite = finite && isfinite(b[k]);
      for (int l = 0; l < R; ++l) {
        finite = finite && isfinite(A[k][l]);
        amax = fmax(amax, fabs(A[k][l]));
      }
    }
    I.resid[iter] = sqrt(nrm);
    if (!finite && st == 0) {
      atomicOr(I.status, ST_NONFINITE);
      st |= ST_NONFINITE;
    }
    x[0] = amax;
  }
  __syncthreads();
  const double amax = x[0];
  if (mode & SOLVE_WRITE_SYSTEM) {
    for (int p = lane; p < R * R; p += 64) A_out[p] = A[p / R][p % R];
    if (lane < R) phi_out[lane] = b[lane];
  }
  if (!(mode & SOLVE_UPDATE)) return;
  if (st != 0) return;  // frozen: keep the last good state
  // LU with partial pivoting on [A | -phi]
  if (lane < R) b[lane] = -b[lane];
  __syncthreads();
  for (int k = 0; k < R; ++k) {
    double v = (lane >= k && lane < R) ? fabs(A[lane][k]) : -1.0;
    int idx = lane;
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(v, off);
      const int oi = __shfl_xor(idx, off);
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
    const int p = idx;
    if (!(v > 1e-300 * amax)) {
      if (lane == 0) flag = 1;
    }
    if (p != k) {
      if (lane < R) {
        const double t0 = A[k][lane];
        A[k][lane] = A[p][lane];
        A[p][lane] = t0;
      }
      if (lane == 0) {
        const double t1 = b[k];
        b[k] = b[p];
        b[p] = t1;
      }
    }
    __syncthreads();
    if (lane > k && lane < R) {
      const double f = A[lane][k] / A[k][k];
      for (int j = k + 1; j < R; ++j) A[lane][j] -= f * A[k][j];
      b[lane] -= f * b[k];
    }
    __syncthreads();
  }
  if (flag) {
    if (lane == 0) atomicOr(I.status, ST_SINGULAR);
    return;
  }
  for (int k = R - 1; k >= 0; --k) {
    if (lane == 0) x[k] = b[k] / A[k][k];
    __syncthreads();
    if (lane < k) b[lane] -= A[lane][k] * x[k];
    __syncthreads();
  }
  if (lane < R) I.r[lane] += x[lane];
  __syncthreads();
  if (lane < nq) {
    const double q = I.r[np + lane];
    I.dec_in[lane] = q;
    I.dec_in[nq + lane] = q - I.rbar[np + lane];
    I.dec_in[2 * nq + lane] = I.rdot[np + lane];
  }
  if ((mode & SOLVE_FINISH) && lane < R) {
    const double rn = I.r[lane];
    I.rdot[lane] = (rn - I.rbar[lane]) / dt;
    I.rbar[lane] = rn;
  }
}

template <typename T>
void launch_solve(const Inst<T>* tab, int nb, int iter, int mode, double* A_out, double* phi_out, hipStream_t s) {
  k_solve<T><<<dim3(1, nb), 64, 0, s>>>(tab, iter, mode, A_out, phi_out);
}
template void launch_solve<float>(const Inst<float>*, int, int, int, double*, double*, hipStream_t);
template void launch_solve<double>(const Inst<double>*, int, int, int, double*, double*, hipStream_t);

}  // namespace nmr
