// Coupled multi-domain step (Sec. 6.8): a core domain and rods whose root-face
// vertex copies are tied to core vertices by zero-length springs of
// stiffness kappa.  Every domain runs its own decoder, cubature, mass terms
// and backpropagation (the domain kernels, with the tie force added to its
// internal force), and writes its own Newton system (eq. system_mat); the
// kernels here add the tie terms and solve the stacked system
//   [A_c'   Cc_1 ... Cc_m] [d_c]     [phi_c']
//   [Cc_1^T A_1'        ] [d_1]  = -[phi_1']
//   [ ...          ...  ] [...]     [ ... ]
// by static condensation onto the core: each rod's block is eliminated on
// its own (k_couple_local, one block per rod), the core's Schur complement
//   S = A_c' - sum_k Cc_k A_k'^-1 Cc_k^T
// is summed over the rods in a fixed order (k_couple_sum) and solved
// (k_couple_core), and each
// rod back-substitutes (k_couple_back).  A_d' and phi_d' are the domain's
// own matrix and residual plus its tie stiffness and tie force.  All
// reduced arithmetic in FP64.  Dense elimination with partial pivoting, as
// in the single-domain solve, with the same pivot threshold.
#include "nmr_internal.h"

namespace nmr {

// ---------------------------------------------------------------------------
// Tie forces and tie blocks, one 64-thread block per rod: lane t owns tie
// DOF pair t (rod DOF dr, core DOF dc); gap = (X + u)_rod - (X + u)_core,
// f = kappa gap is the rod's tie force (dE_tie/du_rod), -f the core's.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_couple_pen(const Inst<T>* __restrict__ mem, CoupleDev cd) {
  const int k = blockIdx.x, lane = threadIdx.x;
  const Inst<T>& C = mem[0];
  const Inst<T>& D = mem[1 + k];
  const int Rc = C.R, Rr = D.R, npc = C.n_p, npr = D.n_p, Cfc = C.Cf, Cfr = D.Cf, ntd = cd.n_td;
  const double dt2 = C.dt * C.dt, kap = cd.kappa;
  __shared__ double Jr[64][NMR_MAX_R + 1], Jc[64][NMR_MAX_R + 1], f[64];
  if (lane < ntd) {
    const int dr = ldg<int>(cd.tie + 2 * (k * ntd + lane)), dc = ldg<int>(cd.tie + 2 * (k * ntd + lane) + 1);
    const double ur = (double)ldg<T>(D.rec + (size_t)dr * Cfr), uc = (double)ldg<T>(C.rec + (size_t)dc * Cfc);
    const double gap = ((double)ldg<T>(D.X + dr) + ur) - ((double)ldg<T>(C.X + dc) + uc);
    const double fv = kap * gap;
    stg<T>(D.pen + dr, (T)fv);
    stg<T>(C.pen + dc, (T)(-fv));
    f[lane] = fv;
    for (int j = 0; j < Rr; ++j)
      Jr[lane][j] = j < npr ? (double)ldg<T>(D.U + (size_t)dr * npr + j) : (double)ldg<T>(D.rec + (size_t)dr * Cfr + 1 + j - npr);
    for (int j = 0; j < Rc; ++j)
      Jc[lane][j] = j < npc ? (double)ldg<T>(C.U + (size_t)dc * npc + j) : (double)ldg<T>(C.rec + (size_t)dc * Cfc + 1 + j - npc);
  }
  __syncthreads();
  double* w = cd.ws + (size_t)k * kCoupleWs;
  for (int e = lane; e < Rr * Rr; e += 64) {
    const int a = e / Rr, b = e - a * Rr;
    double s = 0.0;
    for (int t = 0; t < ntd; ++t) s += Jr[t][a] * Jr[t][b];
    stg<double>(w + CW_PR + a * NMR_MAX_R + b, dt2 * kap * s);
  }
  for (int e = lane; e < Rc * Rc; e += 64) {
    const int a = e / Rc, b = e - a * Rc;
    double s = 0.0;
    for (int t = 0; t < ntd; ++t) s += Jc[t][a] * Jc[t][b];
    stg<double>(w + CW_PC + a * NMR_MAX_R + b, dt2 * kap * s);
  }
  for (int e = lane; e < Rc * Rr; e += 64) {
    const int a = e / Rr, b = e - a * Rr;
    double s = 0.0;
    for (int t = 0; t < ntd; ++t) s += Jc[t][a] * Jr[t][b];
    stg<double>(w + CW_CC + a * NMR_MAX_R + b, -dt2 * kap * s);
  }
  if (lane < Rr) {
    double s = 0.0;
    for (int t = 0; t < ntd; ++t) s += Jr[t][lane] * f[t];
    stg<double>(w + CW_GR + lane, dt2 * s);
  }
  if (lane < Rc) {
    double s = 0.0;
    for (int t = 0; t < ntd; ++t) s += Jc[t][lane] * f[t];
    stg<double>(w + CW_GC + lane, -dt2 * s);
  }
}

// ---------------------------------------------------------------------------
// Gauss-Jordan elimination with partial pivoting (rows swapped in LDS) of
// the n x nc matrix M whose first n columns are the system matrix; on
// return columns n.. hold the solutions.  Pivot: the largest |M_ip| among
// the rows not yet used, ties to the lower row; singular when it is below
// 1e-300 max |M_ij| (j < n).  256 threads, every thread reaches every
// barrier; returns true when singular or not finite.
// ---------------------------------------------------------------------------
constexpr int kLd = 2 * NMR_MAX_R + 2;

__device__ bool gj_solve(double (*M)[kLd], int n, int nc) {
  const int tid = threadIdx.x, lane = tid & 63;
  __shared__ double fac[NMR_MAX_R], s_amax;
  __shared__ int s_piv, s_bad;
  if (tid < 64) {
    double m = 0.0;
    bool fin = true;
    for (int j = 0; j < nc; ++j) {
      const double v = lane < n ? M[lane][j] : 0.0;
      fin = fin && isfinite(v);
      if (j < n) m = fmax(m, fabs(v));
    }
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    const bool all_fin = __all(fin);
    if (lane == 0) {
      s_amax = m;
      s_bad = all_fin ? 0 : 1;
    }
  }
  __syncthreads();
  if (s_bad) return true;
  const double amax = s_amax;
  for (int p = 0; p < n; ++p) {
    if (tid < 64) {
      double key = (lane >= p && lane < n) ? fabs(M[lane][p]) : -1.0;
      int idx = lane;
      for (int o = 32; o > 0; o >>= 1) {
        const double ok = __shfl_xor(key, o);
        const int oi = __shfl_xor(idx, o);
        if (ok > key || (ok == key && oi < idx)) {
          key = ok;
          idx = oi;
        }
      }
      if (lane == 0) {
        s_piv = idx;
        s_bad = !(key > 1e-300 * amax);
      }
    }
    __syncthreads();
    if (s_bad) return true;
    const int q = s_piv;
    if (q != p)
      for (int j = tid; j < nc; j += 256) {
        const double t = M[p][j];
        M[p][j] = M[q][j];
        M[q][j] = t;
      }
    __syncthreads();
    const double piv = M[p][p];
    __syncthreads();
    for (int j = tid; j < nc; j += 256) M[p][j] /= piv;
    if (tid < n) fac[tid] = tid == p ? 0.0 : M[tid][p];
    __syncthreads();
    for (int e = tid; e < n * nc; e += 256) {
      const int i = e / nc, j = e - i * nc;
      if (i != p) M[i][j] = fma(-fac[i], M[p][j], M[i][j]);
    }
    __syncthreads();
  }
  return false;
}

// r += delta (threads j < R), then on the last iteration of the step
// rdot = (r - rbar) / dt and rbar = r; the decoder input (q, q - qbar,
// qdot_bar) of the next iteration
template <typename T>
__device__ void couple_update(const Inst<T>& I, const double* delta, int iter, int mode, double nrm) {
  const int j = threadIdx.x, R = I.R, np = I.n_p, nq = I.n_q;
  const bool fin = mode & SOLVE_FINISH;
  if (j == 0) stg<double>(I.resid + iter, nrm);
  if (j < R) {
    const double r0 = ldg<double>(I.r + j), rb = ldg<double>(I.rbar + j), rd = ldg<double>(I.rdot + j);
    const double rn = r0 + delta[j];
    const double rbn = fin ? rn : rb;
    const double rdn = fin ? (rn - rb) / I.dt : rd;
    stg<double>(I.r + j, rn);
    if (fin) {
      stg<double>(I.rbar + j, rbn);
      stg<double>(I.rdot + j, rdn);
    }
    if (j >= np) {
      stg<double>(I.dec_in + (j - np), rn);
      stg<double>(I.dec_in + nq + (j - np), rn - rbn);
      stg<double>(I.dec_in + 2 * nq + (j - np), rdn);
    }
  }
}

// ---------------------------------------------------------------------------
// Rod k: A' = A_k + Pr, phi' = phi_k + gr; X = A'^-1 [phi', Cc^T]; the
// rod's Schur terms Sc = Cc X[:, 1:], sc = Cc X[:, 0].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_couple_local(const Inst<T>* __restrict__ mem, CoupleDev cd) {
  const int k = blockIdx.x, tid = threadIdx.x;
  const Inst<T>& C = mem[0];
  const Inst<T>& D = mem[1 + k];
  const int Rc = C.R, Rr = D.R, nc = Rr + 1 + Rc;
  double* w = cd.ws + (size_t)k * kCoupleWs;
  __shared__ double M[NMR_MAX_R][kLd];
  for (int e = tid; e < Rr * nc; e += 256) {
    const int i = e / nc, j = e - i * nc;
    double v;
    if (j < Rr) v = ldg<double>(D.sysA + i * Rr + j) + ldg<double>(w + CW_PR + i * NMR_MAX_R + j);
    else if (j == Rr) v = ldg<double>(D.sysphi + i) + ldg<double>(w + CW_GR + i);
    else v = ldg<double>(w + CW_CC + (j - Rr - 1) * NMR_MAX_R + i);
    M[i][j] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int i = 0; i < Rr; ++i) s += M[i][Rr] * M[i][Rr];
    stg<double>(w + CW_NRM, s);
  }
  const bool bad = gj_solve(M, Rr, nc);
  if (bad) {
    if (tid == 0) atomicOr(D.status, ST_SINGULAR);
    return;
  }
  for (int e = tid; e < Rr * (1 + Rc); e += 256) {
    const int i = e / (1 + Rc), j = e - i * (1 + Rc);
    stg<double>(w + CW_X + i * (NMR_MAX_R + 1) + j, M[i][Rr + j]);
  }
  for (int e = tid; e < Rc * (1 + Rc); e += 256) {
    const int a = e / (1 + Rc), j = e - a * (1 + Rc);
    double s = 0.0;
    for (int i = 0; i < Rr; ++i) s += ldg<double>(w + CW_CC + a * NMR_MAX_R + i) * M[i][Rr + j];
    if (j == 0) stg<double>(w + CW_SCV + a, s);
    else stg<double>(w + CW_SC + a * NMR_MAX_R + (j - 1), s);
  }
}

// ---------------------------------------------------------------------------
// Sums over the rods of the core's terms, in fixed order: entry e of
//   [sum_k (Pc_k - Sc_k) (R_c x R_c) | sum_k gc_k (R_c) | sum_k sc_k (R_c) |
//    sum_k |phi'_k|^2]
// 16 entries per block; slice s of 16 threads adds rods s, s + 16, ... and
// the slice sums are added in slice order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_couple_sum(const Inst<T>* __restrict__ mem, CoupleDev cd) {
  const int Rc = mem[0].R, m = cd.n_rods;
  const int ne = Rc * Rc + 2 * Rc + 1;
  const int kk = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const int e = blockIdx.x * 16 + kk;
  __shared__ double part[16][17];
  double acc = 0.0;
  if (e < ne) {
    for (int k = sl; k < m; k += 16) {
      const double* w = cd.ws + (size_t)k * kCoupleWs;
      if (e < Rc * Rc) {
        const int a = e / Rc, b = e - a * Rc;
        acc += ldg<double>(w + CW_PC + a * NMR_MAX_R + b) - ldg<double>(w + CW_SC + a * NMR_MAX_R + b);
      } else if (e < Rc * Rc + Rc) {
        acc += ldg<double>(w + CW_GC + (e - Rc * Rc));
      } else if (e < Rc * Rc + 2 * Rc) {
        acc += ldg<double>(w + CW_SCV + (e - Rc * Rc - Rc));
      } else {
        acc += ldg<double>(w + CW_NRM);
      }
    }
  }
  part[sl][kk] = acc;
  __syncthreads();
  if (sl == 0 && e < ne) {
    double v = part[0][kk];
    for (int q = 1; q < 16; ++q) v += part[q][kk];
    stg<double>(cd.red + e, v);
  }
}

// ---------------------------------------------------------------------------
// Core: members' status (any failure freezes the whole set and is reported
// by every member), S = A_c + sum_k (Pc_k - Sc_k), rhs = -(phi_c + sum_k gc_k)
// + sum_k sc_k (rods added in rod order), S d_c = rhs, core update.  The
// core's recorded residual is the norm of the stacked phi'.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_couple_core(const Inst<T>* __restrict__ mem, CoupleDev cd, int iter,
                                                     int mode) {
  const int tid = threadIdx.x, m = cd.n_rods;
  const Inst<T>& C = mem[0];
  const int Rc = C.R;
  __shared__ int bits;
  __shared__ double M[NMR_MAX_R][kLd];
  __shared__ double phic[NMR_MAX_R], sdel[NMR_MAX_R], snrm;
  if (tid == 0) bits = 0;
  __syncthreads();
  for (int k = tid; k <= m; k += 256) {
    const int st = *gp(mem[k].status);
    if (st) atomicOr(&bits, st);
  }
  __syncthreads();
  if (bits) {
    for (int k = tid; k <= m; k += 256) atomicOr(mem[k].status, bits);
    if (tid == 0) stg<int>(cd.frozen, 1);
    return;
  }
  for (int e = tid; e < Rc * Rc + Rc; e += 256) {
    if (e < Rc * Rc) {
      const int a = e / Rc, b = e - a * Rc;
      M[a][b] = ldg<double>(C.sysA + a * Rc + b) + ldg<double>(cd.red + e);
    } else {
      const int a = e - Rc * Rc;
      const double ph = ldg<double>(C.sysphi + a) + ldg<double>(cd.red + Rc * Rc + a);
      phic[a] = ph;
      M[a][Rc] = -ph + ldg<double>(cd.red + Rc * Rc + Rc + a);
    }
  }
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int a = 0; a < Rc; ++a) s += phic[a] * phic[a];
    snrm = sqrt(s + ldg<double>(cd.red + Rc * Rc + 2 * Rc));
  }
  const bool bad = gj_solve(M, Rc, Rc + 1);
  if (bad) {
    for (int k = tid; k <= m; k += 256) atomicOr(mem[k].status, ST_SINGULAR);
    if (tid == 0) stg<int>(cd.frozen, 1);
    return;
  }
  if (tid < Rc) {
    sdel[tid] = M[tid][Rc];
    stg<double>(cd.dc + tid, M[tid][Rc]);
  }
  if (tid == 0) stg<int>(cd.frozen, 0);
  __syncthreads();
  couple_update(C, sdel, iter, mode, snrm);
}

// Rod k: d_k = -X[:, 0] - X[:, 1:] d_c, rod update.
template <typename T>
__global__ __launch_bounds__(64) void k_couple_back(const Inst<T>* __restrict__ mem, CoupleDev cd, int iter,
                                                    int mode) {
  const int k = blockIdx.x, tid = threadIdx.x;
  if (*gp(cd.frozen)) return;
  const Inst<T>& C = mem[0];
  const Inst<T>& D = mem[1 + k];
  const int Rc = C.R, Rr = D.R;
  const double* w = cd.ws + (size_t)k * kCoupleWs;
  __shared__ double sdel[NMR_MAX_R];
  if (tid < Rr) {
    double v = -ldg<double>(w + CW_X + tid * (NMR_MAX_R + 1));
    for (int b = 0; b < Rc; ++b) v -= ldg<double>(w + CW_X + tid * (NMR_MAX_R + 1) + 1 + b) * ldg<double>(cd.dc + b);
    sdel[tid] = v;
  }
  __syncthreads();
  couple_update(D, sdel, iter, mode, sqrt(ldg<double>(w + CW_NRM)));
}

template <typename T>
void launch_couple_pen(const Inst<T>* mem, const CoupleDev& cd, hipStream_t s) {
  k_couple_pen<T><<<cd.n_rods, 64, 0, s>>>(mem, cd);
}
template <typename T>
void launch_couple_solve(const Inst<T>* mem, const CoupleDev& cd, int iter, int mode, hipStream_t s) {
  k_couple_local<T><<<cd.n_rods, 256, 0, s>>>(mem, cd);
  k_couple_sum<T><<<(NMR_MAX_R * NMR_MAX_R + 2 * NMR_MAX_R + 1 + 15) / 16, 256, 0, s>>>(mem, cd);
  k_couple_core<T><<<1, 256, 0, s>>>(mem, cd, iter, mode);
  k_couple_back<T><<<cd.n_rods, 64, 0, s>>>(mem, cd, iter, mode);
}
template void launch_couple_pen<float>(const Inst<float>*, const CoupleDev&, hipStream_t);
template void launch_couple_pen<double>(const Inst<double>*, const CoupleDev&, hipStream_t);
template void launch_couple_solve<float>(const Inst<float>*, const CoupleDev&, int, int, hipStream_t);
template void launch_couple_solve<double>(const Inst<double>*, const CoupleDev&, int, int, hipStream_t);

}  // namespace nmr
