// Neural cubature training (Sec. 5) on the GPU.
//
// Training data (Sec. 5.1): for every pose r_p the reduced force of every
// element, F[p][e] = Jt_e(r_p)^T f_e(u(r_p)) (R doubles), and its sum over
// the elements f[p] (full quadrature).  The two networks train in alternation
// with full-batch Adam on relative squared losses averaged over the poses:
//   weight net W (the run-time form: softplus after every layer, times a
//   fixed scale): L_W = mean_p |f_p - sum_{j<|C|} w_j(r_p) F[p][C_j]|^2 / |f_p|^2
//   selection net S (two graph convolutions of eq. of the graph convolution,
//   8 channels, sin; element feature = mean of its vertices; FC 8 -> 8 sin,
//   FC 8 -> 1; scores s = e^c softmax over the elements outside C):
//   L_S = mean_p |fb_p - sum_{e not in C} s_e F[p][e]|^2 / |fb_p|^2,
//   fb_p the residual force of the current cubature (eq. of the residual force).
// After each net's epochs the K candidates with the largest score averaged
// over the poses join C.
//
// Every sum runs in a fixed order (block partials added in block order), so
// a run is bitwise repeatable.  All arithmetic in FP64.
//
// Layouts (row-major): F [P][m][R], f and fb [P][R], u [P][N]; selection-net
// vertex features [P][n][8] (H0 [P][n][3]); element adjoints dg [P][m][8];
// parameter vector theta (170): G0 [3][8] (in, out), G1 [8][8] (in, out),
// A1 [8][8] (out, in), a1 [8], A2 [8], a2, c.
#include "train_internal.h"

#include <algorithm>

namespace nmr {

// ---------------------------------------------------------------------------
// rest shape of every tet: B_m = D_m^-1, V = det D_m / 6
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rest_all(const double* X, const int* tets, int m, double* Bm, double* Ve) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= m) return;
  int v[4];
  for (int a = 0; a < 4; ++a) v[a] = ldg<int>(tets + 4 * e + a);
  double D[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) D[i][k] = ldg<double>(X + 3 * v[k + 1] + i) - ldg<double>(X + 3 * v[0] + i);
  const double c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  const double c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  const double c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  const double det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
  const double id = 1.0 / det;
  double B[3][3];  // inverse = adjugate / det
  B[0][0] = c00 * id;
  B[1][0] = c01 * id;
  B[2][0] = c02 * id;
  B[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * id;
  B[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * id;
  B[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * id;
  B[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * id;
  B[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * id;
  B[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * id;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) stg<double>(Bm + 9 * e + 3 * i + j, B[i][j]);
  stg<double>(Ve + e, det / 6.0);
}

void launch_rest_all(const double* X, const int* tets, int m, double* Bm, double* Ve, hipStream_t s) {
  k_rest_all<<<(m + 255) / 256, 256, 0, s>>>(X, tets, m, Bm, Ve);
}

// ---------------------------------------------------------------------------
// training data of one pose
// ---------------------------------------------------------------------------
// u = U p + D(q) in FP64
template <typename T>
__global__ __launch_bounds__(256) void k_pose_u(const T* U, int n_p, const double* r, const T* uD, int N, double* u) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double acc = 0.0;
  for (int k = 0; k < n_p; ++k) acc += (double)ldg<T>(U + (size_t)i * n_p + k) * ldg<double>(r + k);
  stg<double>(u + i, acc + (double)ldg<T>(uD + i));
}

// One thread per tet: neo-Hookean P = mu (F - F^-T) + lam ln J F^-T, vertex
// forces f_a = V P g_a (g_a = row a - 1 of B_m for a >= 1, g_0 = -(g_1 + g_2
// + g_3)), then F_e[r] = sum_{a, i} Jt[3 v_a + i][r] f_a[i] with Jt = [U, J].
template <typename T>
__global__ __launch_bounds__(256) void k_elem_forces(const double* X, const int* tets, const double* Bm,
                                                     const double* Ve, double mu, double lam, int m, const T* U,
                                                     int n_p, const T* J, int n_q, const double* u, double* Fout,
                                                     int* status) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= m) return;
  int v[4];
  for (int a = 0; a < 4; ++a) v[a] = ldg<int>(tets + 4 * e + a);
  double x[4][3];
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 3; ++c) x[a][c] = ldg<double>(X + 3 * v[a] + c) + ldg<double>(u + 3 * v[a] + c);
  double B[3][3];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) B[k][j] = ldg<double>(Bm + 9 * e + 3 * k + j);
  double F[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += (x[k + 1][i] - x[0][i]) * B[k][j];
      F[i][j] = acc;
    }
  const double det = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                     F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                     F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  if (!(det > 0.0)) {
    atomicOr(status, ST_INVERTED);
    for (int r = 0; r < n_p + n_q; ++r) stg<double>(Fout + (size_t)e * (n_p + n_q) + r, 0.0);
    return;
  }
  const double id = 1.0 / det;
  double A[3][3];  // F^-T
  A[0][0] = (F[1][1] * F[2][2] - F[1][2] * F[2][1]) * id;
  A[1][0] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * id;
  A[2][0] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * id;
  A[0][1] = (F[1][2] * F[2][0] - F[1][0] * F[2][2]) * id;
  A[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * id;
  A[2][1] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * id;
  A[0][2] = (F[1][0] * F[2][1] - F[1][1] * F[2][0]) * id;
  A[1][2] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * id;
  A[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * id;
  const double lnJ = log(det);
  const double V = ldg<double>(Ve + e);
  double f[4][3];
  for (int i = 0; i < 3; ++i) {
    double P[3];
    for (int j = 0; j < 3; ++j) P[j] = mu * (F[i][j] - A[i][j]) + lam * lnJ * A[i][j];
    double s0 = 0.0;
    for (int a = 1; a < 4; ++a) {
      f[a][i] = V * (P[0] * B[a - 1][0] + P[1] * B[a - 1][1] + P[2] * B[a - 1][2]);
      s0 += f[a][i];
    }
    f[0][i] = -s0;
  }
  const int R = n_p + n_q;
  for (int r = 0; r < R; ++r) {
    double acc = 0.0;
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) {
        const size_t dof = (size_t)3 * v[a] + i;
        const double jt = r < n_p ? (double)ldg<T>(U + dof * n_p + r) : (double)ldg<T>(J + dof * n_q + (r - n_p));
        acc += jt * f[a][i];
      }
    stg<double>(Fout + (size_t)e * R + r, acc);
  }
}

template <typename T>
void launch_elem_forces(const TrainMesh& tm, const T* U, int n_p, const double* r, const T* uD, const T* J, int n_q,
                        double* u, double* F, int* status, hipStream_t s) {
  k_pose_u<T><<<(tm.N + 255) / 256, 256, 0, s>>>(U, n_p, r, uD, tm.N, u);
  k_elem_forces<T><<<(tm.m + 255) / 256, 256, 0, s>>>(tm.X, tm.tets, tm.Bm, tm.Ve, tm.mu, tm.lam, tm.m, U, n_p, J,
                                                      n_q, u, F, status);
}
template void launch_elem_forces<float>(const TrainMesh&, const float*, int, const double*, const float*,
                                        const float*, int, double*, double*, int*, hipStream_t);
template void launch_elem_forces<double>(const TrainMesh&, const double*, int, const double*, const double*,
                                         const double*, int, double*, double*, int*, hipStream_t);

// ---------------------------------------------------------------------------
// fixed-order block sums of R-vectors: thread t of a 256-thread block holds
// v[0..R); thread r < R of the block gets the sum over t in index order.
// ---------------------------------------------------------------------------
__device__ inline double block_sum_col(double (*sh)[NMR_MAX_R + 1], int R) {
  __syncthreads();
  double s = 0.0;
  if ((int)threadIdx.x < R)
    for (int t = 0; t < 256; ++t) s += sh[t][threadIdx.x];
  return s;
}

// f[p] = sum_e F[p][e] (elements in index order, per thread stride 256)
__global__ __launch_bounds__(256) void k_force_sum(const double* F, int m, int R, double* f) {
  const int p = blockIdx.x, t = threadIdx.x;
  __shared__ double sh[256][NMR_MAX_R + 1];
  double acc[NMR_MAX_R];
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  const double* Fp = F + (size_t)p * m * R;
  for (int e = t; e < m; e += 256)
    for (int r = 0; r < R; ++r) acc[r] += ldg<double>(Fp + (size_t)e * R + r);
  for (int r = 0; r < R; ++r) sh[t][r] = acc[r];
  const double s = block_sum_col(sh, R);
  if (t < R) stg<double>(f + (size_t)p * R + t, s);
}

void launch_force_sum(const double* F, int P, int m, int R, double* f, hipStream_t s) {
  k_force_sum<<<P, 256, 0, s>>>(F, m, R, f);
}

// ---------------------------------------------------------------------------
// weight net: z_{l+1} = softplus(W_l z_l + b_l), w = scale z_L (rows < nC)
// ---------------------------------------------------------------------------
__device__ inline double softplus_d(double x) { return x > 0.0 ? x + log1p(exp(-x)) : log1p(exp(x)); }
__device__ inline double sigmoid_d(double x) { return 0.5 * (1.0 + tanh(0.5 * x)); }

// thread per (output o, pose p): a[p][o] = W[o] . z[p] + b[o]
__global__ __launch_bounds__(256) void k_w_layer(const double* W, const double* b, const double* zin, int win,
                                                 int wout, int nact, int P, double* a, double* z) {
  const int o = blockIdx.x * 64 + (threadIdx.x & 63);
  const int p = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (o >= nact || p >= P) return;
  const double* w = W + (size_t)o * win;
  const double* x = zin + (size_t)p * win;
  double acc = 0.0;
  for (int i = 0; i < win; ++i) acc += ldg<double>(w + i) * ldg<double>(x + i);
  acc += ldg<double>(b + o);
  stg<double>(a + (size_t)p * wout + o, acc);
  stg<double>(z + (size_t)p * wout + o, softplus_d(acc));
}

// Block per pose: res = f - sum_{j<nC} scale z_L[j] F[C_j]; per-pose loss
// |res|^2 / |f|^2 / P.  mode 0: also the output adjoint
// delta_L[j] = scale coef (F[C_j] . res) sigmoid(a_L[j]), coef = -2 / (P |f|^2)
// (zero for j >= nC); mode 1: res is stored as the residual force fb.
__global__ __launch_bounds__(256) void k_w_res(const double* F, const double* f, const int* C, int nC, int c_max,
                                               int m, int R, const double* aL, const double* zL, double scale, int P,
                                               int mode, double* res_out, double* loss, double* deltaL) {
  const int p = blockIdx.x, t = threadIdx.x;
  __shared__ double sh[256][NMR_MAX_R + 1];
  __shared__ double res[NMR_MAX_R];
  __shared__ double nf_s;
  const double* Fp = F + (size_t)p * m * R;
  double acc[NMR_MAX_R];
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  for (int j = t; j < nC; j += 256) {
    const double w = scale * ldg<double>(zL + (size_t)p * c_max + j);
    const double* row = Fp + (size_t)ldg<int>(C + j) * R;
    for (int r = 0; r < R; ++r) acc[r] += w * ldg<double>(row + r);
  }
  for (int r = 0; r < R; ++r) sh[t][r] = acc[r];
  const double s = block_sum_col(sh, R);
  if (t < R) res[t] = ldg<double>(f + (size_t)p * R + t) - s;
  __syncthreads();
  if (t == 0) {
    double nf = 0.0, rr = 0.0;
    for (int r = 0; r < R; ++r) {
      const double fr = ldg<double>(f + (size_t)p * R + r);
      nf += fr * fr;
      rr += res[r] * res[r];
    }
    nf_s = nf;
    stg<double>(loss + p, rr / nf / P);
  }
  __syncthreads();
  if (mode == 1) {
    if (t < R) stg<double>(res_out + (size_t)p * R + t, res[t]);
    return;
  }
  const double coef = -2.0 / (P * nf_s);
  for (int j = t; j < c_max; j += 256) {
    double d = 0.0;
    if (j < nC) {
      const double* row = Fp + (size_t)ldg<int>(C + j) * R;
      double dot = 0.0;
      for (int r = 0; r < R; ++r) dot += ldg<double>(row + r) * res[r];
      d = scale * (coef * dot) * sigmoid_d(ldg<double>(aL + (size_t)p * c_max + j));
    }
    stg<double>(deltaL + (size_t)p * c_max + j, d);
  }
}

// delta_in[p][i] = sigmoid(a_in[p][i]) sum_{o<nact} W[o][i] delta_out[p][o]
__global__ __launch_bounds__(256) void k_w_back(const double* W, const double* dout, int wout, int nact,
                                                const double* ain, int win, int P, double* din) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int p = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= win || p >= P) return;
  double acc = 0.0;
  for (int o = 0; o < nact; ++o) acc += ldg<double>(W + (size_t)o * win + i) * ldg<double>(dout + (size_t)p * wout + o);
  stg<double>(din + (size_t)p * win + i, acc * sigmoid_d(ldg<double>(ain + (size_t)p * win + i)));
}

// gW[o][i] = sum_p delta[p][o] z[p][i] (i < win), gb[o] = sum_p delta[p][o]
// (column i = win of a z extended by ones).  Block: a 64 x 64 output tile,
// 16 x 16 threads with 4 x 4 outputs each; poses staged 32 at a time in LDS
// and added in pose order.
__global__ __launch_bounds__(256) void k_w_grad(const double* delta, int wout, const double* zin, int win, int P,
                                                double* gW, double* gb) {
  __shared__ double sD[32][64], sZ[32][65];
  const int o0 = blockIdx.y * 64, i0 = blockIdx.x * 64, t = threadIdx.x, ty = t / 16, tx = t % 16;
  double acc[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int p0 = 0; p0 < P; p0 += 32) {
    for (int k = t; k < 32 * 64; k += 256) {
      const int pp = k / 64, c = k % 64, p = p0 + pp;
      const int o = o0 + c, i = i0 + c;
      sD[pp][c] = (p < P && o < wout) ? ldg<double>(delta + (size_t)p * wout + o) : 0.0;
      sZ[pp][c] = (p < P && i < win) ? ldg<double>(zin + (size_t)p * win + i) : (p < P && i == win) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int np = min(32, P - p0);
    for (int pp = 0; pp < np; ++pp) {
      double d[4], z[4];
      for (int a = 0; a < 4; ++a) d[a] = sD[pp][ty * 4 + a];
      for (int b = 0; b < 4; ++b) z[b] = sZ[pp][tx * 4 + b];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] += d[a] * z[b];
    }
    __syncthreads();
  }
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const int o = o0 + ty * 4 + a, i = i0 + tx * 4 + b;
      if (o >= wout) continue;
      if (i < win) stg<double>(gW + (size_t)o * win + i, acc[a][b]);
      else if (i == win) stg<double>(gb + o, acc[a][b]);
    }
}

// out = sum_p in[p] (poses in order)
__global__ void k_sum_poses(const double* in, int P, double* out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int p = 0; p < P; ++p) s += ldg<double>(in + p);
  stg<double>(out, s);
}

// Adam (Kingma and Ba 2015), c1 = 1 - b1^t, c2 = 1 - b2^t
__global__ __launch_bounds__(256) void k_adam(double* x, const double* g, double* mo, double* ve, long long n,
                                              double lr, double b1, double b2, double eps, double c1, double c2) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double gi = ldg<double>(g + i);
  const double m = b1 * ldg<double>(mo + i) + (1.0 - b1) * gi;
  const double v = b2 * ldg<double>(ve + i) + (1.0 - b2) * (gi * gi);
  stg<double>(mo + i, m);
  stg<double>(ve + i, v);
  stg<double>(x + i, ldg<double>(x + i) - lr * (m / c1) / (sqrt(v / c2) + eps));
}

void launch_wnet_epoch(const WNetDev& w, const TrainData& td, int nC, int mode, hipStream_t s) {
  const int L = w.L;
  const int P = td.P;
  // forward
  const double* zin = td.r;
  for (int l = 0; l < L; ++l) {
    const int nact = l == L - 1 ? nC : w.width[l + 1];
    dim3 grid((nact + 63) / 64, (P + 3) / 4);
    k_w_layer<<<grid, 256, 0, s>>>(w.x + w.Woff[l], w.x + w.boff[l], zin, w.width[l], w.width[l + 1], nact, P,
                                   w.a[l], w.z[l]);
    zin = w.z[l];
  }
  const int cmax = w.width[L];
  k_w_res<<<P, 256, 0, s>>>(td.F, td.f, td.C, nC, cmax, td.m, td.R, w.a[L - 1], w.z[L - 1], w.scale, P, mode,
                            td.fb, td.loss_p, w.d[L - 1]);
  if (mode == 1) return;
  k_sum_poses<<<1, 64, 0, s>>>(td.loss_p, P, w.loss_out);
  // backward: gradient of layer l from delta[l] and z[l - 1] (r for l = 0)
  for (int l = L - 1; l >= 0; --l) {
    const int wout = w.width[l + 1], win = w.width[l];
    const double* zl = l == 0 ? td.r : w.z[l - 1];
    dim3 gg((win + 1 + 63) / 64, (wout + 63) / 64);
    k_w_grad<<<gg, 256, 0, s>>>(w.d[l], wout, zl, win, P, w.g + w.Woff[l], w.g + w.boff[l]);
    if (l > 0) {
      const int nact = l == L - 1 ? nC : wout;
      dim3 grid((win + 63) / 64, (P + 3) / 4);
      k_w_back<<<grid, 256, 0, s>>>(w.x + w.Woff[l], w.d[l], wout, nact, w.a[l - 1], win, P, w.d[l - 1]);
    }
  }
}

void launch_adam(double* x, const double* g, double* m, double* v, long long n, double lr, double b1, double b2,
                 double eps, double c1, double c2, hipStream_t s) {
  k_adam<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

// ---------------------------------------------------------------------------
// selection net
// ---------------------------------------------------------------------------
#define SB 256                // vertices per block
#define SBE NMR_TRAIN_SBE     // elements per block
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Blocks renumbered per XCD (xcd_block): neighbouring vertex and element
// blocks, which gather each other's features, share an L2.
// (b, pc) = (vertex or element block, pose of the chunk).

// the 8 channels of one vertex or element, stored and loaded back to back
__device__ inline void store8(double* dst, const double (&v)[8]) {
  for (int k = 0; k < 4; ++k) stg<double2>(dst + 2 * k, make_double2(v[2 * k], v[2 * k + 1]));
}
__device__ inline void load8(const double* src, double (&v)[8]) {
  for (int k = 0; k < 4; ++k) {
    const double2 x = ldg<double2>(src + 2 * k);
    v[2 * k] = x.x;
    v[2 * k + 1] = x.y;
  }
}

// first convolution: H0 = sum_j A_ij u_j (3), P1 = H0 G0, X1 = sin P1
__global__ __launch_bounds__(SB) void k_gcn1(SNetDev sd) {
  int b, pc;
  xcd_block(b, pc);
  const int v = b * SB + threadIdx.x;
  if (v >= sd.n) return;
  const double* u = sd.u + (size_t)(sd.p0 + pc) * 3 * sd.n;
  double h[3] = {0.0, 0.0, 0.0};
  const int j0 = ldg<int>(sd.g_ptr + v), j1 = ldg<int>(sd.g_ptr + v + 1);
  for (int k = j0; k < j1; ++k) {
    const int j = ldg<int>(sd.g_idx + k);
    const double a = ldg<double>(sd.g_val + k);
    for (int c = 0; c < 3; ++c) h[c] += a * ldg<double>(u + 3 * j + c);
  }
  const size_t vi = (size_t)pc * sd.n + v;
  for (int c = 0; c < 3; ++c) stg<double>(sd.H0 + 3 * vi + c, h[c]);
  const double* G0 = sd.theta;
  double P[8], X[8];
  for (int o = 0; o < 8; ++o) {
    double acc = 0.0;
    for (int c = 0; c < 3; ++c) acc += h[c] * ldg<double>(G0 + 8 * c + o);
    P[o] = acc;
    X[o] = sin(acc);
  }
  store8(sd.P1 + 8 * vi, P);
  store8(sd.X1 + 8 * vi, X);
}

// second convolution: H1 = sum_j A_ij X1_j (8), P2 = H1 G1, X2 = sin P2
__global__ __launch_bounds__(SB) void k_gcn2(SNetDev sd) {
  int b, pc;
  xcd_block(b, pc);
  const int v = b * SB + threadIdx.x;
  if (v >= sd.n) return;
  const double* X1 = sd.X1 + (size_t)pc * 8 * sd.n;
  double h[8];
  for (int c = 0; c < 8; ++c) h[c] = 0.0;
  const int j0 = ldg<int>(sd.g_ptr + v), j1 = ldg<int>(sd.g_ptr + v + 1);
  for (int k = j0; k < j1; ++k) {
    const int j = ldg<int>(sd.g_idx + k);
    const double a = ldg<double>(sd.g_val + k);
    double x[8];
    load8(X1 + 8 * j, x);
    for (int c = 0; c < 8; ++c) h[c] += a * x[c];
  }
  const size_t vi = (size_t)pc * sd.n + v;
  store8(sd.H1 + 8 * vi, h);
  const double* G1 = sd.theta + 24;
  double P[8], X[8];
  for (int o = 0; o < 8; ++o) {
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) acc += h[c] * ldg<double>(G1 + 8 * c + o);
    P[o] = acc;
    X[o] = sin(acc);
  }
  store8(sd.P2 + 8 * vi, P);
  store8(sd.X2 + 8 * vi, X);
}

// element head: g = mean of the 4 vertices' X2, Q = A1 g + a1, Y = sin Q, z = A2 . Y + a2
__device__ inline double elem_head(const SNetDev& sd, int pc, int e, double (&g)[8], double (&Q)[8], double (&Y)[8]) {
  const double* X2 = sd.X2 + (size_t)pc * 8 * sd.n;
  for (int c = 0; c < 8; ++c) g[c] = 0.0;
  for (int a = 0; a < 4; ++a) {
    const int v = ldg<int>(sd.tets + 4 * e + a);
    double x[8];
    load8(X2 + 8 * v, x);
    for (int c = 0; c < 8; ++c) g[c] += x[c];
  }
  for (int c = 0; c < 8; ++c) g[c] = g[c] / 4.0;
  const double* A1 = sd.theta + 88;
  const double* a1 = sd.theta + 152;
  const double* A2 = sd.theta + 160;
  double z = 0.0;
  for (int o = 0; o < 8; ++o) {
    double acc = 0.0;
    for (int i = 0; i < 8; ++i) acc += ldg<double>(A1 + 8 * o + i) * g[i];
    Q[o] = acc + ldg<double>(a1 + o);
    Y[o] = sin(Q[o]);
    z += Y[o] * ldg<double>(A2 + o);
  }
  return z + ldg<double>(sd.theta + 168);
}

// LDS row stride of an F tile: R + 1 columns (R forces and one more value),
// rounded up to an odd number of doubles so that rows fall in different banks
__device__ __host__ inline int tile_ld(int R) { return (R + 1) | 1; }

// Stage the block's F rows [SBE][R] of pose p in LDS with coalesced loads.
__device__ inline void load_F_tile(const SNetDev& sd, int p, int e0, double* tile) {
  const int R = sd.R, ld = tile_ld(R);
  const int ne = min(SBE, sd.m - e0);
  const double* src = sd.F + ((size_t)p * sd.m + e0) * R;
  // element and column of flat index k, advanced by SBE without a division
  int k = threadIdx.x, e = k / R, c = k - e * R;
  const int de = SBE / R, dc = SBE - de * R;
  for (; k < ne * R; k += SBE) {
    tile[e * ld + c] = ldg<double>(src + k);
    e += de;
    c += dc;
    if (c >= R) {
      c -= R;
      ++e;
    }
  }
}

// Forward over the elements, block b of pose p: z (stored), block max M_b of
// the candidates' z, and with w_e = exp(z_e - M_b): S_b = sum w_e and
// V_b = sum w_e F[p][e]; partial layout [P][nbe][R + 2] = (V_b, S_b, M_b).
__global__ __launch_bounds__(SBE) void k_sfwd_elem(SNetDev sd) {
  extern __shared__ double lds[];
  int b, pc;
  xcd_block(b, pc);
  const int p = sd.p0 + pc, t = threadIdx.x, R = sd.R, ld = tile_ld(R);
  const int e0 = b * SBE, e = e0 + t;
  double* tile = lds;                    // [SBE][ld], column R = w
  __shared__ double red[SBE];
  __shared__ double part[SBE / 32][NMR_MAX_R + 2];
  load_F_tile(sd, p, e0, tile);
  bool cand = false;
  double z = -INFINITY;
  if (e < sd.m) {
    double g[8], Q[8], Y[8];
    z = elem_head(sd, pc, e, g, Q, Y);
    stg<double>(sd.z + (size_t)p * sd.m + e, z);
    cand = ldg<int>(sd.inC + e) == 0;
  }
  red[t] = cand ? z : -INFINITY;
  __syncthreads();
  for (int h = SBE / 2; h > 0; h >>= 1) {
    if (t < h) red[t] = fmax(red[t], red[t + h]);
    __syncthreads();
  }
  const double Mb = red[0];
  const double w = cand ? exp(z - Mb) : 0.0;
  tile[t * ld + R] = w;
  __syncthreads();
  // slices of 32 elements: thread (slice, col) sums its column
  const int col = t % 32, sl = t / 32;
  if (col <= R) {
    const int ne = min(SBE, sd.m - e0);
    double acc = 0.0;
    for (int k = sl * 32; k < min(ne, sl * 32 + 32); ++k) {
      const double wk = tile[k * ld + R];
      acc += col == R ? wk : wk * tile[k * ld + col];
    }
    part[sl][col] = acc;
  }
  __syncthreads();
  if (t <= R) {
    double s = 0.0;
    for (int k = 0; k < SBE / 32; ++k) s += part[k][t];
    stg<double>(sd.pf + ((size_t)pc * sd.nbe + b) * (R + 2) + t, s);
  }
  if (t == 0) stg<double>(sd.pf + ((size_t)pc * sd.nbe + b) * (R + 2) + R + 1, Mb);
}

// Per pose: M = max M_b, S = sum S_b e^{M_b - M}, V likewise; res = fb - e^c V / S,
// loss_p = |res|^2 / |fb|^2 / P, coef = -2 / (P |fb|^2), qbar = coef (V / S) . res.
// 256 threads: 8 slices of the blocks per column, slice sums added in order.
__global__ __launch_bounds__(256) void k_scombine(SNetDev sd) {
  const int pc = blockIdx.x, p = sd.p0 + pc, t = threadIdx.x, R = sd.R;
  __shared__ double part[8][NMR_MAX_R + 1];
  __shared__ double col[NMR_MAX_R + 1];
  __shared__ double red[256];
  const double* pf = sd.pf + (size_t)pc * sd.nbe * (R + 2);
  double M = -INFINITY;
  for (int b = t; b < sd.nbe; b += 256) M = fmax(M, ldg<double>(pf + (size_t)b * (R + 2) + R + 1));
  red[t] = M;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] = fmax(red[t], red[t + h]);
    __syncthreads();
  }
  M = red[0];
  const int c = t % 32, sl = t / 32;
  if (c <= R) {
    const int per = (sd.nbe + 7) / 8;
    double s = 0.0;
    for (int b = sl * per; b < min(sd.nbe, sl * per + per); ++b) {
      const double Mb = ldg<double>(pf + (size_t)b * (R + 2) + R + 1);
      if (Mb == -INFINITY) continue;
      s += ldg<double>(pf + (size_t)b * (R + 2) + c) * exp(Mb - M);
    }
    part[sl][c] = s;
  }
  __syncthreads();
  if (t <= R) {
    double s = 0.0;
    for (int k = 0; k < 8; ++k) s += part[k][t];
    col[t] = s;
  }
  __syncthreads();
  if (t == 0) {
    const double S = col[R];
    const double ec = exp(ldg<double>(sd.theta + 169));
    double nf = 0.0, rr = 0.0, q = 0.0;
    double* res = sd.res + (size_t)p * R;
    for (int r = 0; r < R; ++r) {
      const double fb = ldg<double>(sd.fb + (size_t)p * R + r);
      const double pr = col[r] / S;
      const double rv = fb - ec * pr;
      stg<double>(res + r, rv);
      nf += fb * fb;
      rr += rv * rv;
      q += pr * rv;
    }
    const double coef = -2.0 / (sd.P * nf);
    double* ps = sd.pstat + (size_t)p * 8;
    stg<double>(ps + 0, M);
    stg<double>(ps + 1, S);
    stg<double>(ps + 2, coef);
    stg<double>(ps + 3, coef * q);       // qbar
    stg<double>(ps + 4, ec * coef * q);  // dL/dc of this pose
    stg<double>(sd.loss_p + p, rr / nf / sd.P);
  }
}

// Backward over the elements: ds_e = coef F[p][e] . res, dz = s (ds - qbar),
// dQ = dz A2 cos Q, dg = A1^T dQ (stored); block partials of the element-head
// gradients, layout [P][nbe][81] = (A1 [8][8], a1, A2, a2) in theta order.
__global__ __launch_bounds__(SBE) void k_sbwd_elem(SNetDev sd) {
  extern __shared__ double lds[];
  int b, pc;
  xcd_block(b, pc);
  const int p = sd.p0 + pc, t = threadIdx.x, R = sd.R, ld = tile_ld(R);
  const int e0 = b * SBE, e = e0 + t;
  double* tile = lds;                        // [SBE][ld]
  double(*sv)[25] = (double(*)[25])lds;      // after the dot products: dz, dQ (8), g (8), Y (8)
  __shared__ double cmb[2][16][16];
  __shared__ double res[NMR_MAX_R];
  load_F_tile(sd, p, e0, tile);
  if (t < R) res[t] = ldg<double>(sd.res + (size_t)p * R + t);
  __syncthreads();
  double dz = 0.0, dQ[8], g[8], Y[8];
  for (int c = 0; c < 8; ++c) dQ[c] = g[c] = Y[c] = 0.0;
  if (e < sd.m) {
    // the head again, without the logit (the forward pass stored it)
    const double* X2 = sd.X2 + (size_t)pc * 8 * sd.n;
    for (int a = 0; a < 4; ++a) {
      const int v = ldg<int>(sd.tets + 4 * e + a);
      double x[8];
      load8(X2 + 8 * v, x);
      for (int c = 0; c < 8; ++c) g[c] += x[c];
    }
    for (int c = 0; c < 8; ++c) g[c] = g[c] / 4.0;
    double cQ[8];
    for (int o = 0; o < 8; ++o) {
      double acc = 0.0;
      for (int i = 0; i < 8; ++i) acc += ldg<double>(sd.theta + 88 + 8 * o + i) * g[i];
      sincos(acc + ldg<double>(sd.theta + 152 + o), &Y[o], &cQ[o]);
    }
    const double z = ldg<double>(sd.z + (size_t)p * sd.m + e);
    const double* ps = sd.pstat + (size_t)p * 8;
    double dg[8];
    for (int c = 0; c < 8; ++c) dg[c] = 0.0;
    if (ldg<int>(sd.inC + e) == 0) {
      const double M = ldg<double>(ps + 0), S = ldg<double>(ps + 1), coef = ldg<double>(ps + 2),
                   qbar = ldg<double>(ps + 3);
      const double s = exp(ldg<double>(sd.theta + 169)) * (exp(z - M) / S);
      double dot = 0.0;
      for (int r = 0; r < R; ++r) dot += tile[t * ld + r] * res[r];
      dz = s * (coef * dot - qbar);
      const double* A1 = sd.theta + 88;
      const double* A2 = sd.theta + 160;
      for (int o = 0; o < 8; ++o) dQ[o] = dz * ldg<double>(A2 + o) * cQ[o];
      for (int i = 0; i < 8; ++i) {
        double acc = 0.0;
        for (int o = 0; o < 8; ++o) acc += dQ[o] * ldg<double>(A1 + 8 * o + i);
        dg[i] = acc;
      }
    }
    store8(sd.dg + ((size_t)pc * sd.m + e) * 8, dg);
  }
  __syncthreads();  // every dot product has read the tile
  sv[t][0] = dz;
  for (int c = 0; c < 8; ++c) {
    sv[t][1 + c] = dQ[c];
    sv[t][9 + c] = g[c];
    sv[t][17 + c] = Y[c];
  }
  __syncthreads();
  // The 81 head gradients as two outer-product sums over the block's elements
  // on the FP64 matrix cores: with a_e = [dQ (8), dz, 0 ...] and
  // b_e = [g (8), Y (8)], D = sum_e a_e b_e^T holds dA1 (rows 0-7, columns 0-7)
  // and dA2 (row 8, columns 8-15); D2 = sum_e a_e e_0^T holds da1 and da2
  // (column 0).  Each wave takes its 64 elements four at a time
  // (v_mfma_f64_16x16x4: A[m][k] from lane m + 16 k, B[k][n] from lane n + 16 k;
  // item q of lane l is D[4 q + l / 16][l % 16]); wave partials are added in
  // wave order.
  {
    const int wave = t >> 6, lane = t & 63, col = lane & 15, kk = lane >> 4;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
    const double b2 = col == 0 ? 1.0 : 0.0;
    for (int step = 0; step < 16; ++step) {
      const int row = wave * 64 + step * 4 + kk;
      const double a = col < 8 ? sv[row][1 + col] : col == 8 ? sv[row][0] : 0.0;
      const double bb = col < 8 ? sv[row][9 + col] : sv[row][17 + (col - 8)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b2, acc2, 0, 0, 0);
    }
    for (int w = 0; w < SBE / 64; ++w) {
      if (wave == w)
        for (int q = 0; q < 4; ++q) {
          const int rr = 4 * q + kk;
          cmb[0][rr][col] = (w == 0 ? 0.0 : cmb[0][rr][col]) + acc[q];
          cmb[1][rr][col] = (w == 0 ? 0.0 : cmb[1][rr][col]) + acc2[q];
        }
      __syncthreads();
    }
  }
  if (t < 81) {
    const double v = t < 64 ? cmb[0][t / 8][t % 8]             // dA1[o][i]
                   : t < 72 ? cmb[1][t - 64][0]                 // da1[o]
                   : t < 80 ? cmb[0][8][8 + (t - 72)]           // dA2[i]
                            : cmb[1][8][0];                     // da2
    stg<double>(sd.pe + ((size_t)pc * sd.nbe + b) * 81 + t, v);
  }
}

// Second convolution backward, per vertex: dX2 = sum over incident tets of
// dg / 4, dP2 = dX2 cos P2, T2 = dP2 G1^T (stored); partials of
// dG1[i][o] = sum_v H1_i dP2_o, layout [P][nbv][64].
__global__ __launch_bounds__(SB) void k_sbwd_v2(SNetDev sd) {
  int b, p;  // p: pose of the chunk
  xcd_block(b, p);
  const int t = threadIdx.x;
  const int v = b * SB + t;
  __shared__ double sv[SB][17];  // H1 (8), dP2 (8), padded
  __shared__ double part[4][64];
  double h[8], d[8];
  for (int c = 0; c < 8; ++c) h[c] = d[c] = 0.0;
  if (v < sd.n) {
    const size_t vi = (size_t)p * sd.n + v;
    const double* dg = sd.dg + (size_t)p * sd.m * 8;
    double dx[8];
    for (int c = 0; c < 8; ++c) dx[c] = 0.0;
    const int k0 = ldg<int>(sd.vt_ptr + v), k1 = ldg<int>(sd.vt_ptr + v + 1);
    for (int k = k0; k < k1; ++k) {
      const int e = ldg<int>(sd.vt_tet + k);
      double x[8];
      load8(dg + (size_t)e * 8, x);
      for (int c = 0; c < 8; ++c) dx[c] += x[c] / 4.0;
    }
    for (int c = 0; c < 8; ++c) {
      h[c] = ldg<double>(sd.H1 + 8 * vi + c);
      d[c] = dx[c] * cos(ldg<double>(sd.P2 + 8 * vi + c));
    }
    const double* G1 = sd.theta + 24;
    double T[8];
    for (int i = 0; i < 8; ++i) {
      double acc = 0.0;
      for (int o = 0; o < 8; ++o) acc += d[o] * ldg<double>(G1 + 8 * i + o);
      T[i] = acc;
    }
    store8(sd.T2 + 8 * vi, T);
  }
  for (int c = 0; c < 8; ++c) {
    sv[t][c] = h[c];
    sv[t][8 + c] = d[c];
  }
  __syncthreads();
  {
    const int j = t % 64, sl = t / 64, i = j / 8, o = j % 8;
    double acc = 0.0;
    for (int k = sl * 64; k < sl * 64 + 64; ++k) acc += sv[k][i] * sv[k][8 + o];
    part[sl][j] = acc;
  }
  __syncthreads();
  if (t < 64)
    stg<double>(sd.pv2 + ((size_t)p * sd.nbv + b) * 64 + t, ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t]);
}

// First convolution backward, per vertex: dX1 = sum_j A_ij T2_j,
// dP1 = dX1 cos P1; partials of dG0[c][o] = sum_v H0_c dP1_o, [P][nbv][24].
__global__ __launch_bounds__(SB) void k_sbwd_v1(SNetDev sd) {
  int b, p;  // p: pose of the chunk
  xcd_block(b, p);
  const int t = threadIdx.x;
  const int v = b * SB + t;
  __shared__ double sv[SB][11];  // H0 (3), dP1 (8)
  __shared__ double part[8][24];
  double h[3] = {0.0, 0.0, 0.0}, d[8];
  for (int c = 0; c < 8; ++c) d[c] = 0.0;
  if (v < sd.n) {
    const size_t vi = (size_t)p * sd.n + v;
    const double* T2 = sd.T2 + (size_t)p * 8 * sd.n;
    double dx[8];
    for (int c = 0; c < 8; ++c) dx[c] = 0.0;
    const int j0 = ldg<int>(sd.g_ptr + v), j1 = ldg<int>(sd.g_ptr + v + 1);
    for (int k = j0; k < j1; ++k) {
      const int j = ldg<int>(sd.g_idx + k);
      const double a = ldg<double>(sd.g_val + k);
      double x[8];
      load8(T2 + 8 * j, x);
      for (int c = 0; c < 8; ++c) dx[c] += a * x[c];
    }
    for (int c = 0; c < 8; ++c) d[c] = dx[c] * cos(ldg<double>(sd.P1 + 8 * vi + c));
    for (int c = 0; c < 3; ++c) h[c] = ldg<double>(sd.H0 + 3 * vi + c);
  }
  for (int c = 0; c < 3; ++c) sv[t][c] = h[c];
  for (int c = 0; c < 8; ++c) sv[t][3 + c] = d[c];
  __syncthreads();
  if (t < 192) {
    const int j = t % 24, sl = t / 24, c = j / 8, o = j % 8;
    double acc = 0.0;
    for (int k = sl * 32; k < sl * 32 + 32; ++k) acc += sv[k][c] * sv[k][3 + o];
    part[sl][j] = acc;
  }
  __syncthreads();
  if (t < 24) {
    double s = 0.0;
    for (int k = 0; k < 8; ++k) s += part[k][t];
    stg<double>(sd.pv1 + ((size_t)p * sd.nbv + b) * 24 + t, s);
  }
}

// Per pose: the 170 gradient entries from the block partials: 4 slices of
// the blocks per entry (blocks in order within a slice, slices in order).
__global__ __launch_bounds__(1024) void k_sred_pose(SNetDev sd) {
  const int pc = blockIdx.x, p = sd.p0 + pc, t = threadIdx.x;
  const int k = t % 256, sl = t / 256;
  __shared__ double part[4][170];
  if (k < 170) {
    double s = 0.0;
    if (k < 169) {
      const bool vert = k < 88;
      const int nb = vert ? sd.nbv : sd.nbe;
      const int per = (nb + 3) / 4, b0 = sl * per, b1 = min(nb, b0 + per);
      const double* src = k < 24 ? sd.pv1 + (size_t)pc * sd.nbv * 24 + k
                        : k < 88 ? sd.pv2 + (size_t)pc * sd.nbv * 64 + (k - 24)
                                 : sd.pe + (size_t)pc * sd.nbe * 81 + (k - 88);
      const int ld = k < 24 ? 24 : k < 88 ? 64 : 81;
      for (int b = b0; b < b1; ++b) s += ldg<double>(src + (size_t)b * ld);
    } else if (sl == 0) {
      s = ldg<double>(sd.pstat + (size_t)p * 8 + 4);
    }
    part[sl][k] = s;
  }
  __syncthreads();
  if (t < 170) stg<double>(sd.gpose + (size_t)p * 170 + t, ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t]);
}

// grad[k] = sum_p gpose[p][k] (block k < 170) and the loss (block 170):
// each of 256 threads adds every 256th pose in order, then a fixed tree.
__global__ __launch_bounds__(256) void k_sred_all(SNetDev sd) {
  const int k = blockIdx.x, t = threadIdx.x;
  __shared__ double red[256];
  double s = 0.0;
  for (int p = t; p < sd.P; p += 256)
    s += k < 170 ? ldg<double>(sd.gpose + (size_t)p * 170 + k) : ldg<double>(sd.loss_p + p);
  red[t] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) stg<double>(k < 170 ? sd.grad + k : sd.loss_out, red[0]);
}

static size_t tile_bytes(int R) { return (size_t)SBE * tile_ld(R) * sizeof(double); }
static size_t bwd_bytes(int R) { return std::max(tile_bytes(R), (size_t)SBE * 25 * sizeof(double)); }

// Poses go through in chunks of sd.nc (the last one shorter): the per-pose
// intermediates of a chunk ([nc][n][8] features, [nc][m][8] adjoints) stay
// small enough to be re-read from the caches rather than from HBM.
static void forward_chunk(SNetDev c, hipStream_t s) {
  dim3 gv(c.nbv, c.nc), ge(c.nbe, c.nc);
  k_gcn1<<<gv, SB, 0, s>>>(c);
  k_gcn2<<<gv, SB, 0, s>>>(c);
  k_sfwd_elem<<<ge, SBE, tile_bytes(c.R), s>>>(c);
  k_scombine<<<c.nc, 256, 0, s>>>(c);
}

void launch_snet_forward(const SNetDev& sd, hipStream_t s) {
  for (int p0 = 0; p0 < sd.P; p0 += sd.nc) {
    SNetDev c = sd;
    c.p0 = p0;
    c.nc = std::min(sd.nc, sd.P - p0);
    forward_chunk(c, s);
  }
}

void launch_snet_epoch(const SNetDev& sd, hipStream_t s) {
  for (int p0 = 0; p0 < sd.P; p0 += sd.nc) {
    SNetDev c = sd;
    c.p0 = p0;
    c.nc = std::min(sd.nc, sd.P - p0);
    forward_chunk(c, s);
    dim3 gv(c.nbv, c.nc), ge(c.nbe, c.nc);
    k_sbwd_elem<<<ge, SBE, bwd_bytes(c.R), s>>>(c);
    k_sbwd_v2<<<gv, SB, 0, s>>>(c);
    k_sbwd_v1<<<gv, SB, 0, s>>>(c);
    k_sred_pose<<<c.nc, 1024, 0, s>>>(c);
  }
  k_sred_all<<<171, 256, 0, s>>>(sd);
}

void launch_snet_elem(const SNetDev& sd, int backward, hipStream_t s) {
  for (int p0 = 0; p0 < sd.P; p0 += sd.nc) {
    SNetDev c = sd;
    c.p0 = p0;
    c.nc = std::min(sd.nc, sd.P - p0);
    dim3 ge(c.nbe, c.nc);
    if (backward)
      k_sbwd_elem<<<ge, SBE, bwd_bytes(c.R), s>>>(c);
    else
      k_sfwd_elem<<<ge, SBE, tile_bytes(c.R), s>>>(c);
  }
}

// ---------------------------------------------------------------------------
// selection of K new cubature elements
// ---------------------------------------------------------------------------
// mean[e] = (1/P) sum_p e^c exp(z[p][e] - M_p) / S_p for candidates, -inf otherwise
__global__ __launch_bounds__(256) void k_smean(SNetDev sd, double* mean) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= sd.m) return;
  if (ldg<int>(sd.inC + e)) {
    stg<double>(mean + e, -INFINITY);
    return;
  }
  const double ec = exp(ldg<double>(sd.theta + 169));
  double acc = 0.0;
  for (int p = 0; p < sd.P; ++p) {
    const double M = ldg<double>(sd.pstat + (size_t)p * 8), S = ldg<double>(sd.pstat + (size_t)p * 8 + 1);
    const double s = ec * (exp(ldg<double>(sd.z + (size_t)p * sd.m + e) - M) / S);
    acc += s / sd.P;
  }
  stg<double>(mean + e, acc);
}

// better(a, b): larger value, then lower index
__device__ inline bool better(double va, int ia, double vb, int ib) { return va > vb || (va == vb && ia < ib); }

// One block: K rounds of the block-wide best candidate; each joins C.
__global__ __launch_bounds__(1024) void k_topk(double* mean, int m, int K, int* inC, int* C, int nC) {
  const int t = threadIdx.x;
  __shared__ double bv[1024];
  __shared__ int bi[1024];
  for (int k = 0; k < K; ++k) {
    double v = -INFINITY;
    int idx = 0x7fffffff;
    for (int e = t; e < m; e += 1024) {
      const double x = mean[e];
      if (x != -INFINITY && better(x, e, v, idx)) {
        v = x;
        idx = e;
      }
    }
    bv[t] = v;
    bi[t] = idx;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
      if (t < h && better(bv[t + h], bi[t + h], bv[t], bi[t])) {
        bv[t] = bv[t + h];
        bi[t] = bi[t + h];
      }
      __syncthreads();
    }
    if (t == 0) {
      const int e = bi[0];
      if (e >= 0 && e < m) {
        C[nC + k] = e;
        inC[e] = 1;
        mean[e] = -INFINITY;
      } else {
        C[nC + k] = -1;  // no finite candidate score: reported by the host
      }
    }
    __syncthreads();
  }
}

void launch_select(const SNetDev& sd, double* mean, int K, int* inC, int* C, int nC, hipStream_t s) {
  k_smean<<<(sd.m + 255) / 256, 256, 0, s>>>(sd, mean);
  k_topk<<<1, 1024, 0, s>>>(mean, sd.m, K, inC, C, nC);
}

// ---------------------------------------------------------------------------
// farthest-point (Voronoi) samples of the element centroids from element 0.
// Centroid and distance in the order ((x0 + x1) + x2) + x3 / 4 and
// sqrt((dx^2 + dy^2) + dz^2) without contraction; ties to the lower index.
// ---------------------------------------------------------------------------
__device__ inline void centroid(const double* X, const int* tets, int e, double (&c)[3]) {
#pragma clang fp contract(off)
  for (int d = 0; d < 3; ++d) {
    double s = ldg<double>(X + 3 * ldg<int>(tets + 4 * e) + d);
    for (int a = 1; a < 4; ++a) s = s + ldg<double>(X + 3 * ldg<int>(tets + 4 * e + a) + d);
    c[d] = s / 4.0;
  }
}

__device__ inline double cdist(const double (&a)[3], const double (&b)[3]) {
#pragma clang fp contract(off)
  const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return sqrt((dx * dx + dy * dy) + dz * dz);
}

__global__ __launch_bounds__(1024) void k_fps(const double* X, const int* tets, int m, int k, double* dist, int* C,
                                              int* inC) {
  const int t = threadIdx.x;
  __shared__ double bv[1024];
  __shared__ int bi[1024];
  __shared__ int last;
  if (t == 0) {
    last = 0;
    C[0] = 0;
    inC[0] = 1;
  }
  __syncthreads();
  for (int s = 1; s <= k; ++s) {
    double cl[3];
    centroid(X, tets, last, cl);
    double v = -1.0;
    int idx = 0x7fffffff;
    for (int e = t; e < m; e += 1024) {
      double ce[3];
      centroid(X, tets, e, ce);
      const double d = cdist(ce, cl);
      const double dn = s == 1 ? d : fmin(dist[e], d);
      dist[e] = dn;
      if (better(dn, e, v, idx)) {
        v = dn;
        idx = e;
      }
    }
    if (s == k) break;
    bv[t] = v;
    bi[t] = idx;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
      if (t < h && better(bv[t + h], bi[t + h], bv[t], bi[t])) {
        bv[t] = bv[t + h];
        bi[t] = bi[t + h];
      }
      __syncthreads();
    }
    if (t == 0) {
      const int e = bi[0];
      if (e >= 0 && e < m) {
        last = e;
        C[s] = e;
        inC[e] = 1;
      } else {
        last = 0;   // non-finite distances: reported by the host
        C[s] = -1;
      }
    }
    __syncthreads();
  }
}
void launch_fps(const double* X, const int* tets, int m, int k, double* dist, int* C, int* inC, hipStream_t s) {
  k_fps<<<1, 1024, 0, s>>>(X, tets, m, k, dist, C, inC);
}

}  // namespace nmr
