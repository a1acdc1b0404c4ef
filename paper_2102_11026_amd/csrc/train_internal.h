// Internal declarations of the neural cubature training kernels (train.hip),
// kept apart from the simulator's declarations in nmr_internal.h.
#pragma once

#include "nmr_internal.h"

#define NMR_TRAIN_SBE 128  // elements per block of the selection net's element passes

namespace nmr {

// Mesh of every tet in FP64 (rest shape computed on the device).
struct TrainMesh {
  int n, N, m;
  const double* X;       // [n][3]
  const int* tets;       // [m][4]
  const double* Bm;      // [m][3][3] D_m^-1
  const double* Ve;      // [m] rest volume
  double mu, lam;
};
// Poses, training data and the cubature set.
struct TrainData {
  int P, R, m;
  const double* r;       // [P][R] poses
  const double* F;       // [P][m][R] per-element reduced forces
  const double* f;       // [P][R] full-quadrature reduced force
  double* fb;            // [P][R] residual force of the current cubature
  const int* C;          // [c_max] cubature elements in joining order
  double* loss_p;        // [P] per-pose loss terms
};
// Weight net under training: parameters x = [W_0, b_0, ..., W_{L-1}, b_{L-1}]
// (the last layer with c_max rows), gradient g, activations per layer.
struct WNetDev {
  int L;
  int width[NMR_MAX_LAYERS + 1];
  size_t Woff[NMR_MAX_LAYERS], boff[NMR_MAX_LAYERS];
  double scale;
  double* x;
  double* g;
  double* a[NMR_MAX_LAYERS];  // [P][width[l + 1]] pre-activations
  double* z[NMR_MAX_LAYERS];  // [P][width[l + 1]] outputs
  double* d[NMR_MAX_LAYERS];  // [P][width[l + 1]] adjoints of the pre-activations
  double* loss_out;           // where the epoch's loss is written
};
// Selection net under training.  Poses run in chunks of nc starting at p0:
// arrays marked "chunk" hold the poses of one chunk, the others every pose.
struct SNetDev {
  int n, m, R, P, nbv, nbe;
  int p0, nc;
  const double* u;                     // [P][n][3]
  const int *g_ptr, *g_idx;            // one-ring CSR, self included
  const double* g_val;                 // 1 / sqrt(d_i d_j)
  const int *vt_ptr, *vt_tet;          // vertex -> incident tets
  const int* tets;                     // [m][4]
  const int* inC;                      // [m] 1: in the cubature set
  const double* theta;                 // [170]
  const double* F;                     // [P][m][R]
  const double* fb;                    // [P][R]
  double *H0, *P1, *X1, *H1, *P2, *X2, *T2;  // chunk [nc][n][3 or 8]
  double* z;                           // [P][m] logits
  double* pf;                          // chunk [nc][nbe][R + 2] forward partials
  double* pstat;                       // [P][8]: M, S, coef, qbar, dL/dc
  double* res;                         // [P][R]
  double* loss_p;                      // [P]
  double* dg;                          // chunk [nc][m][8]
  double *pe, *pv2, *pv1;              // chunk gradient partials [nc][nbe][81], [nc][nbv][64], [nc][nbv][24]
  double* gpose;                       // [P][170]
  double* grad;                        // [170]
  double* loss_out;
};
void launch_rest_all(const double* X, const int* tets, int m, double* Bm, double* Ve, hipStream_t s);
template <typename T>
void launch_elem_forces(const TrainMesh& tm, const T* U, int n_p, const double* r, const T* uD, const T* J, int n_q,
                        double* u, double* F, int* status, hipStream_t s);
void launch_force_sum(const double* F, int P, int m, int R, double* f, hipStream_t s);
void launch_wnet_epoch(const WNetDev& w, const TrainData& td, int nC, int mode, hipStream_t s);
void launch_adam(double* x, const double* g, double* m, double* v, long long n, double lr, double b1, double b2,
                 double eps, double c1, double c2, hipStream_t s);
void launch_snet_forward(const SNetDev& sd, hipStream_t s);
void launch_snet_epoch(const SNetDev& sd, hipStream_t s);
void launch_snet_elem(const SNetDev& sd, int backward, hipStream_t s);  // the element pass alone
void launch_select(const SNetDev& sd, double* mean, int K, int* inC, int* C, int nC, hipStream_t s);
void launch_fps(const double* X, const int* tets, int m, int k, double* dist, int* C, int* inC, hipStream_t s);

}  // namespace nmr
