// Internal declarations of libnmr (not part of the C ABI).
//
// Data layout in HBM, per instance (all row-major):
//   dec_in  [3][n_q] f64     q, dq = q - qbar, qdot_bar fed to the decoder
//   act     [2][Cp][Wmax]    post-activation jets, channel-major, ping-pong
//   pre[l]  [Cb][m_l]        hidden pre-activations kept for backpropagation:
//                            channel 0 = value, 1 + j = tangent along e_j
//   fold    [Cf][m_{L-1}]    last hidden layer folded to output channels
//   rec     [N][Cf]          one record per DOF: u, J (n_q), dJ (n_q), Hdd
//   seed    [N]              P a, the backpropagation seed
//   zb      [2][Cb][Wmax]    adjoints of the hidden layers, ping-pong
//   frame   [N]              u of the frame decoded last
// Jet channels of the forward pass (multicomplex units taken to the h -> 0
// limit, i.e. each component stored divided by h^order):
//   0 value, 1 along dq (i2 = i3), 2 along qdot_bar (i4), 3 along (dq, dq),
//   4 + j along e_j (i1), 4 + n_q + j (e_j, dq), 4 + 2 n_q + j (e_j, qdot_bar),
//   4 + 3 n_q + j (e_j, dq, dq).
// Output channels (rec and fold): 0 value, 1 + j  J e_j,
//   1 + n_q + j  dJ e_j = S(e_j,dq,dq) + 3 H(e_j,dq) - dt H(e_j,qdot_bar),
//   1 + 2 n_q  Hdd.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <type_traits>

#define NMR_MAX_LAYERS 16
#define NMR_MAX_R 32
#define NMR_WPAD 32  // every layer width is padded to a multiple of this

typedef __hip_bfloat16 bf16_t;

namespace nmr {

enum { ACT_IDENTITY = 0, ACT_TANH = 1, ACT_ELU = 2, ACT_SIN = 3 };
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16 = 2 };
enum { ST_OK = 0, ST_INVERTED = 1, ST_SINGULAR = 2, ST_NONFINITE = 4 };

inline int pad_to(int x, int m) { return (x + m - 1) / m * m; }

// Device copy of a decoder.  Weights are zero-padded to [out_p][in_p]
// (widths padded to NMR_WPAD) in the decoder's weight type; biases in the
// activation type.
struct DecoderDev {
  int L;
  int act;
  int prec;
  int w[NMR_MAX_LAYERS + 1];   // true widths
  int wp[NMR_MAX_LAYERS + 1];  // padded widths
  const void* W[NMR_MAX_LAYERS];
  const void* b[NMR_MAX_LAYERS];
  const void* WT[NMR_MAX_LAYERS];  // hidden layers: W^T, [in_p][out_p]
};

// Everything a kernel needs to know about one instance.  T = float for the
// FP32 / BF16 forms, double for the FP64 form.  One copy lives in device
// memory per instance; batched launches take an array of them and select
// the instance with blockIdx.y.
template <typename T>
struct Inst {
  int active;              // 0: an empty slot of a pool; every kernel returns at once
  int trimmed;             // 1: fictitious force dropped (dJ = H.(dq - dt qdot), Hdd = 0)
  int fd;                  // 1: derivatives by recursive central differences of step fd_h
  double fd_h;
  int N, n, n_p, n_q, R, n_cub;
  int Cp, Cb, Cf;          // padded channel counts: forward, backward, output
  int Np;                  // N padded to NMR_WPAD
  int n_mblk, n_cblk, n_bblk;  // partial-sum blocks: mass, cubature, bwd-out
  int cub_per_blk;
  double dt, mu, lam, g[3];
  // state
  double* r;
  double* rbar;
  double* rdot;
  double* dec_in;          // [3][n_q]
  double* resid;           // [max_iters]
  int* status;             // sticky failure bits
  // mesh and problem constants
  const T* X;              // [N] rest positions per DOF
  const T* mass;           // [N]
  const T* keep;           // [N] 1 - pinned
  const T* U;              // [N][n_p]
  const int* cub_v;        // [n_cub][4]
  const T* cub_Bm;         // [n_cub][9]
  const T* cub_Ve;         // [n_cub]
  const int* csr_ptr;      // [n + 1] vertex -> (slot, corner) of cubature tets
  const int* csr_ent;      // [4 n_cub], value = 4 * slot + corner
  T* cub_w;                // [n_cub] current weights
  // cubature sources (Newton path: rec / U; API path: caller arrays)
  const T* cu_u; int cu_u_ld;
  const T* cu_Ja; int cu_Ja_ld; int cu_na;
  const T* cu_Jb; int cu_Jb_ld; int cu_nb;
  const T* cu_w;
  // decoder workspaces
  T* act0;
  T* act1;
  T* pre[NMR_MAX_LAYERS];
  T* fold;
  T* rec;
  T* seed;
  T* zb0;
  T* zb1;
  T* fe;                   // [n_cub][12] weighted element forces
  double* part_cub;        // [n_cblk][R*R + R]
  double* part_mass;       // [n_mblk][R*R + R*n_q + R + n_p]
  double* part_bwd;        // [n_bblk][K_last]
  double* part_filt;       // [ceil(N / 256)][n_p][Cf] (n_p > 0): partials of U^T rec
  double* sum_cub;         // [R*R + R]
  double* sum_mass;        // [R*R + R*n_q + R + n_p]
  double* Bq;              // [n_q][n_q] a . H, column j from perturbation j
  double* JTa;             // [n_q]
  T* frame;                // [N] u = U p + D(q) of the frame decoded last
  // coupled sets only (null elsewhere): the tie force of this domain [N],
  // added to f_int in the residual and the backpropagation seed, and the
  // domain's own Newton system written for the coupled solve
  T* pen;
  double* sysA;            // [R][R]
  double* sysphi;          // [R]
  // Gram-folded Newton path (n_p == 0): with the linear output layer W_L and
  // the constant lumped mass, Jt^T M Jt = F_J^T Gam F_J etc. over the folded
  // activations F; only the DOFs of cubature tets are decoded per iteration
  int gram;                // 1: this table entry runs the Gram path
  int n_gblk;              // Gram partial blocks (kGramKParts x K / 16)
  const int* cdofs;        // [n_cdofs] sorted DOFs touched by cubature tets
  int n_cdofs;
  int n_sblk;              // sparse backprop blocks over cdofs (128 rows each)
  const double* Gam;       // [K][K] W_L^T diag(m keep) W_L
  const double* gam;       // [K]    W_L^T (keep * c), c_i = -dt^2 m_i g_(i mod 3)
  // weight net (optional)
  int wn_L;
  int wn_w[NMR_MAX_LAYERS + 1];
  const T* wn_W[NMR_MAX_LAYERS];
  const T* wn_b[NMR_MAX_LAYERS];
  double wn_scale;
  T* wn_buf;               // [2][max width]
  int wn_maxw;
};

// Every device buffer lives in global memory, but pointers read out of an
// Inst table reach the compiler as generic (flat) pointers.  Flat accesses
// also count against the LDS wait counter, so a kernel mixing them with LDS
// work waits for both; these casts make the access a global one.
#define NMR_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ inline const NMR_GLOBAL T* gp(const T* p) {
  return (const NMR_GLOBAL T*)p;
}
template <typename T>
__device__ inline NMR_GLOBAL T* gpw(T* p) {
  return (NMR_GLOBAL T*)p;
}
// Uniform values (kernel arguments, fields of an Inst table entry) that a
// kernel needs are forced into scalar registers at this point: the compiler
// otherwise sinks each scalar load below the early-exit branches, which
// turns one round trip into a chain of dependent ones.
template <typename V>
__device__ inline void in_sgpr(V v) {
  asm volatile("" ::"s"(v));
}
template <typename... A>
__device__ inline void load_now(A... a) {  // by value: every load is made at the call
  (in_sgpr(a), ...);
}

// load / store a V at p through a global pointer.  HIP's vector structs
// (float4, double4, int4, ...) cannot be copied from an address-space
// qualified reference, so they move through a raw vector of the same size
// and alignment.
template <typename V>
struct raw_of {
  typedef unsigned int type __attribute__((ext_vector_type(sizeof(V) / 4), aligned(alignof(V))));
};
template <typename V, typename T>
__device__ inline V ldg(const T* p) {
  if constexpr (std::is_scalar<V>::value) {
    static_assert(std::is_same<V, typename std::remove_cv<T>::type>::value, "scalar loads take the pointee type");
    return *(const NMR_GLOBAL V*)p;
  } else {
    static_assert(sizeof(V) % 4 == 0, "vector loads move whole dwords");
    typedef typename raw_of<V>::type R;
    const R r = *(const NMR_GLOBAL R*)p;
    V v;
    __builtin_memcpy(&v, &r, sizeof(V));
    return v;
  }
}
template <typename V, typename T>
__device__ inline void stg(T* p, V v) {
  if constexpr (std::is_scalar<V>::value || sizeof(V) < 4) {  // scalars, and 2-byte types such as __bf16
    static_assert(std::is_same<V, T>::value, "scalar stores take the pointee type");
    *(NMR_GLOBAL V*)p = v;
  } else {
    typedef typename raw_of<V>::type R;
    R r;
    __builtin_memcpy(&r, &v, sizeof(V));
    *(NMR_GLOBAL R*)p = r;
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  The block (x, y) of a 2-D grid is renumbered so that each XCD takes a
// contiguous run of the logical blocks b + gridDim.x pc, i.e. whole rows of
// the grid: (b, pc) = the logical block's (x, y).
__device__ inline void xcd_block(int& b, int& pc) {
  const int total = gridDim.x * gridDim.y, lin = blockIdx.y * gridDim.x + blockIdx.x;
  const int per = total / 8, rem = total % 8, x = lin % 8, i = lin / 8;
  const int L = x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
  b = L % gridDim.x;
  pc = L / gridDim.x;
}

// f_int[i] = sum of the weighted element forces at DOF i (fixed CSR order)
template <typename T>
__device__ inline double fint_at(const Inst<T>& I, int i) {
  const int v = i / 3, c = i - 3 * v;
  double f = 0.0;
  const int p0 = ldg<int>(I.csr_ptr + v), p1 = ldg<int>(I.csr_ptr + v + 1);
  for (int p = p0; p < p1; ++p) {
    const int ent = ldg<int>(I.csr_ent + p);
    f += (double)ldg<T>(I.fe + (size_t)(ent >> 2) * 12 + 3 * (ent & 3) + c);
  }
  return f;
}

// ---- fixed-order sums of the cubature and mass partials ------------------
// Launches of many instances merge m consecutive blocks of tets into one
// cubature block (fewer, longer blocks); the sums read ceil(n_cblk / m)
// cubature partials.
// (and 8 for a launch of few instances with at least 4096 blocks of tets: a
// large mesh, whose sums would otherwise read thousands of partials)
inline int cubature_merge(int nb, int max_cblk) { return nb >= 64 ? 8 : nb >= 16 ? 4 : max_cblk >= 4096 ? 8 : 1; }

// Block bx of instance by takes 16 entries; 16 slices of 16 threads add every
// sixteenth partial, then the 16 slice sums are added in slice order.
template <typename T>
__device__ __forceinline__ void sums_block(const Inst<T>* __restrict__ tab, int bx, int by, int cub_m) {
  const Inst<T>& I = tab[by];
  load_now(I.active, I.R, I.n_q, I.n_p, I.n_cblk, I.gram, I.n_gblk, I.n_mblk, I.part_cub, I.part_mass, I.sum_cub,
           I.sum_mass);
  if (!I.active) return;
  const int R = I.R;
  const int Ec = R * R + R;
  const int Em = R * R + R * I.n_q + R + I.n_p;
  const int kk = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const int e = bx * 16 + kk;
  __shared__ double part[16][17];
  double acc = 0.0;
  if (e < Ec) {
    const double* src = I.part_cub + e;
    const int nc = (I.n_cblk + cub_m - 1) / cub_m;
#pragma unroll 4
    for (int b = sl; b < nc; b += 16) acc += ldg<double>(src + (size_t)b * Ec);
  } else if (e < Ec + Em) {
    const double* src = I.part_mass + (e - Ec);
    const int nb = I.gram ? I.n_gblk : I.n_mblk;
#pragma unroll 4
    for (int b = sl; b < nb; b += 16) acc += ldg<double>(src + (size_t)b * Em);
  }
  part[sl][kk] = acc;
  __syncthreads();
  if (sl == 0) {
    double v = part[0][kk];
    for (int q = 1; q < 16; ++q) v += part[q][kk];
    if (e < Ec) stg<double>(I.sum_cub + e, v);
    else if (e < Ec + Em) stg<double>(I.sum_mass + e - Ec, v);
  }
}

// ---- tile configurations of the hidden-layer launches (decoder.hip) ----
// ib instances per block (stacked instances share the weight tile); mr
// 16-row tiles per wave (mr > 1: tall tiles, one wave per instance over the
// whole K); jg (forward, ib = mr = 1): the jet columns of a row tile split
// into groups of three perturbations, one block each.  ib == 0: the rule.
struct TileCfg {
  int ib, mr, jg = 0;
};
// jet-group blocks: below this many (row tile, instance) blocks
static constexpr int kJetGroupBlocks = 192;
// K parts of a 16-row block of the Gram terms: each part is a block of its
// own with its own mass and backpropagation partials
static constexpr int kGramKParts = 2;
TileCfg tile_rule(const DecoderDev& d, int l, int nb, int cols, bool fd, bool f64, bool fwd);
bool tile_eligible(const DecoderDev& d, int l, int nb, int cols, bool fd, bool f64, bool fwd, TileCfg c);
// eligible configurations of hidden layer l (at most 6), the rule's among them
int tile_candidates(const DecoderDev& d, int l, int nb, int cols, bool fd, bool f64, bool fwd, TileCfg* out);

// ---- launchers (decoder.hip) -------------------------------------------
template <typename T>
void launch_fwd_hidden(const DecoderDev& d, int l, const Inst<T>* tab, int nb, int max_cp, bool fd, TileCfg cfg,
                       hipStream_t s);
// same_rows: every instance of the table decodes the same rows (the same
// cubature DOFs on the Gram path, or all N rows of one N)
template <typename T>
void launch_fwd_out(const DecoderDev& d, const Inst<T>* tab, int nb, int max_np, int max_cf, bool same_rows,
                    const int* rows, hipStream_t s);
template <typename T>
void launch_filter(const Inst<T>* tab, int nb, int max_n, int add_up, hipStream_t s);
template <typename T>
void launch_bwd_out(const DecoderDev& d, const Inst<T>* tab, int nb, int max_bblk, hipStream_t s);
// the partial sums and the output-layer backpropagation in one launch (Gram
// path, where the seed needs only the element forces)
template <typename T>
void launch_sums_bwd_out(const DecoderDev& d, const Inst<T>* tab, int nb, int max_entries, int max_sblk,
                         int max_cblk, hipStream_t s);
// the Gram path's output-layer backpropagation of instances that all decode
// `rows` (device, nrows ids), batched so each weight row serves several
// (FP32 / BF16; same bits as launch_bwd_out)
template <typename T>
void launch_bwd_out_batch(const DecoderDev& d, const Inst<T>* tab, int nb, const int* rows, int nrows,
                          hipStream_t s);
template <typename T>
void launch_bwd_reduce(const DecoderDev& d, const Inst<T>* tab, int nb, hipStream_t s);
template <typename T>
void launch_bwd_hidden(const DecoderDev& d, int l, const Inst<T>* tab, int nb, int cb, bool fd, TileCfg cfg,
                       hipStream_t s);
template <typename T>
void launch_unpack(const Inst<T>* tab, T* u, T* J, T* dJ, T* Hdd, int N, hipStream_t s);
// the frame's displacement from the forward pass just run: Gram path, the
// value channel of the folded activations through every row of the output
// layer; direct path, the value channel of the records (filtered, U p added)
template <typename T>
void launch_frame(const DecoderDev& d, const Inst<T>* tab, int nb, int max_n, hipStream_t s);
// the same for a group whose every member runs the Gram path, as one GEMM
// with the instances as columns (FP32 / BF16; FP64 falls back to the above)
template <typename T>
void launch_frame_batch(const DecoderDev& d, const Inst<T>* tab, int nb, int max_n, hipStream_t s);

// ---- launchers (sim.hip) -----------------------------------------------
template <typename T>
void launch_rest_shape(const double* X, const int* tets, int m, const int* cub_ids, int n_cub,
                       const int* vt_ptr, const int* vt_ent, int n, double rho,
                       T* cub_Bm, T* cub_Ve, T* mass, double* Ve_tmp, hipStream_t s);
template <typename T>
void launch_step_begin(const Inst<T>* tab, int nb, int mode, int max_cub, hipStream_t s);
// max_r: the largest R in the launch (sizes the kernel's per-tet work)
template <typename T>
void launch_cubature(const Inst<T>* tab, int nb, int max_cblk, int max_r, hipStream_t s);
// the cubature pass and the Gram kernel in one launch (Gram path)
template <typename T>
void launch_cub_gram(const Inst<T>* tab, int nb, int max_cblk, int max_gblk, int K, int nq, hipStream_t s);
template <typename T>
void launch_mass(const Inst<T>* tab, int nb, int max_mblk, int R, int nq, hipStream_t s);
template <typename T>
void launch_seed_from_a(const Inst<T>* tab, const T* a, int nb, int max_mblk, hipStream_t s);
template <typename T>
void launch_sums(const Inst<T>* tab, int nb, int max_entries, int max_cblk, hipStream_t s);
template <typename T>
void launch_solve(const Inst<T>* tab, int nb, int iter, int mode, double* A_out, double* phi_out,
                  hipStream_t s);
template <typename T>
void launch_fint(const Inst<T>* tab, T* f_int, int N, hipStream_t s);
template <typename T>
void launch_gram(const Inst<T>* tab, int nb, int max_gblk, int K, int nq, hipStream_t s);
template <typename T>
void launch_gram_setup(const void* W, int prec, int K, const T* mass, const T* keep, int N, double dt,
                       const double* g, double* Gam, double* gam, hipStream_t s);

// solve modes (SOLVE_WRITE_INST: the system goes to the entry's sysA / sysphi)
enum { SOLVE_UPDATE = 1, SOLVE_FINISH = 2, SOLVE_WRITE_SYSTEM = 4, SOLVE_WRITE_INST = 8 };

// ---- coupled sets (couple.hip) -----------------------------------------
// Member 0 is the core, member 1 + k rod k; rod k's ties are n_td DOF pairs
// (rod DOF, core DOF).  Per-rod FP64 workspace of kCoupleWs doubles, laid
// out with row stride NMR_MAX_R:
//   Pr [R_r][R_r]   dt^2 kappa Jt_r,T^T Jt_r,T       (rod tie stiffness)
//   gr [R_r]        dt^2 Jt_r,T^T f_r                (rod tie force)
//   Pc [R_c][R_c]   dt^2 kappa Jt_c,T^T Jt_c,T       (core tie stiffness)
//   gc [R_c]        dt^2 Jt_c,T^T f_c
//   Cc [R_c][R_r]   -dt^2 kappa Jt_c,T^T Jt_r,T      (core-rod block)
//   X  [R_r][1+R_c] A'^-1 [phi', Cc^T]               (local solve)
//   Sc [R_c][R_c]   Cc X[:, 1:],  sc [R_c]  Cc X[:, 0]
//   nrm2            |phi'_r|^2
enum {
  CW_PR = 0,
  CW_GR = CW_PR + NMR_MAX_R * NMR_MAX_R,
  CW_PC = CW_GR + NMR_MAX_R,
  CW_GC = CW_PC + NMR_MAX_R * NMR_MAX_R,
  CW_CC = CW_GC + NMR_MAX_R,
  CW_X = CW_CC + NMR_MAX_R * NMR_MAX_R,
  CW_SC = CW_X + NMR_MAX_R * (NMR_MAX_R + 1),
  CW_SCV = CW_SC + NMR_MAX_R * NMR_MAX_R,
  CW_NRM = CW_SCV + NMR_MAX_R,
  kCoupleWs = CW_NRM + 8
};
struct CoupleDev {
  int n_rods, n_td;      // rods, tie DOFs per rod (<= 64)
  double kappa;
  const int* tie;        // [n_rods][n_td][2]
  double* ws;            // [n_rods][kCoupleWs]
  double* dc;            // [NMR_MAX_R] core update of the iteration
  double* red;           // [R_c^2 + 2 R_c + 1] sums over the rods (k_couple_sum)
  int* frozen;           // 1: a member has failed, nothing is updated
};
template <typename T>
void launch_couple_pen(const Inst<T>* mem, const CoupleDev& cd, hipStream_t s);
template <typename T>
void launch_couple_solve(const Inst<T>* mem, const CoupleDev& cd, int iter, int mode, hipStream_t s);
// step-begin modes
enum { BEGIN_STEP = 0, BEGIN_SYSTEM = 1 };

}  // namespace nmr
