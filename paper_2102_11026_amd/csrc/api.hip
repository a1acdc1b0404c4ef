// C ABI of libnmr (include/nmr.h): contexts, decoders, instances, HIP-graph
// capture of whole time steps, and the hot-path entry points.  The per-step
// work is a fixed sequence of kernel launches (decoder jets, output layer,
// cubature, mass terms, sums, backpropagation, solve), captured once per
// (instance set, Newton iteration count) and replayed with one
// hipGraphLaunch per step.
#include "nmr_internal.h"
#include "train_internal.h"
#include "nmr.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace nmr;

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                                  \
  do {                                                                                             \
    hipError_t e_ = (x);                                                                           \
    if (e_ != hipSuccess) return fail(NMR_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CHK(x)                 \
  do {                         \
    int c_ = (x);              \
    if (c_ != NMR_OK) return c_; \
  } while (0)

namespace {

struct DevMem {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
};

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

int dalloc(DevMem& m, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) return NMR_OK;
  void* p = nullptr;
  if (hipMalloc(&p, round256(bytes)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(NMR_ERR_OOM, "hipMalloc failed");
  }
  // the zero fill runs on the null stream; a context stream the library
  // created is non-blocking, so wait for it here, before any kernel on that
  // stream may write the buffer
  if (hipMemset(p, 0, round256(bytes)) != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess) {
    (void)hipFree(p);
    return fail(NMR_ERR_DEVICE, "hipMemset failed");
  }
  m.ptrs.push_back(p);
  m.bytes += round256(bytes);
  *out = p;
  return NMR_OK;
}

template <typename P>
int dalloc_t(DevMem& m, size_t count, P** out) {
  void* p;
  int rc = dalloc(m, count * sizeof(P), &p);
  *out = static_cast<P*>(p);
  return rc;
}

uint16_t f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  std::vector<void*> tabs;  // device tables owned by this entry
};

}  // namespace

struct nmr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t cap = nullptr;
  size_t budget = 0;
  size_t used = 0;
  std::map<std::vector<nmr_inst*>, std::map<int, GraphEntry>> many_graphs;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int tile_mode = NMR_TILES_RULE, tile_ib = 1, tile_mr = 1;
  int tile_epoch = 0;  // bumped when the mode changes (pools recapture)
  // autotuned choices by (forward, m_in, m_out, cols, n_inst, prec, fd)
  std::map<std::array<int, 7>, nmr_tile_choice> tuned;
};

struct nmr_decoder {
  nmr_ctx* ctx = nullptr;
  DecoderDev d{};
  DevMem mem;
  int refs = 1;  // the creator's reference
  bool charged = false;
  // Gram matrices of the output layer (Gram-folded path) by mesh: instances of
  // one decoder on the same mesh, mass, pins, time step and gravity share them
  std::map<uint64_t, std::pair<double*, double*>> gram_cache;
  DevMem gram_mem;
};

struct nmr_inst {
  nmr_ctx* ctx = nullptr;
  nmr_decoder* dec = nullptr;
  int prec = PREC_FP32;
  int N = 0, n = 0, n_p = 0, n_q = 0, R = 0, n_cub = 0;
  int Cp = 0, Cb = 0, Cf = 0, n_mblk = 0, n_cblk = 0, n_bblk = 0;
  int gram = 0, n_cdofs = 0, n_sblk = 0;
  std::vector<int> cdofs;  // host copy of the decoded rows of the Gram path
  int fd = 0;  // central-difference derivatives
  size_t bytes = 0;
  DevMem mem;
  void* tab = nullptr;      // Inst<T> on the device
  void* api_tab = nullptr;  // scratch Inst<T> for the caller-array entry points
  std::vector<unsigned char> host;  // host copy of the Inst<T>
  std::map<int, hipGraphExec_t> step_graphs;
  double* A_scratch = nullptr;
  nmr_pool* pool = nullptr;  // the pool this instance is attached to, if any
  int pool_slot = -1;
  int coupled_refs = 0;      // coupled sets this instance is a member of
  int m = 0;                 // tets of the mesh
  std::vector<double> Xh;    // host copies of the rest positions and tets
  std::vector<int32_t> tets_h;  // (the training data covers every tet)
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
static const int kMaxIters = 64;

static int set_device(nmr_ctx* c) {
  HIPCHK(hipSetDevice(c->device));
  return NMR_OK;
}

template <typename T>
static Inst<T>& host_inst(nmr_inst* in) {
  return *reinterpret_cast<Inst<T>*>(in->host.data());
}

static bool is_f64(const nmr_inst* in) { return in->prec == PREC_FP64; }

static void drop_many_graphs(nmr_ctx* c, nmr_inst* in) {
  for (auto it = c->many_graphs.begin(); it != c->many_graphs.end();) {
    if (in == nullptr || std::find(it->first.begin(), it->first.end(), in) != it->first.end()) {
      for (auto& kv : it->second) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        for (void* p : kv.second.tabs) (void)hipFree(p);
      }
      it = c->many_graphs.erase(it);
    } else {
      ++it;
    }
  }
}

static int check_mlp(const nmr_mlp_desc* d, int min_layers, const char* what) {
  if (!d) return fail(NMR_ERR_ARG, std::string(what) + ": missing description");
  if (d->n_layers < min_layers || d->n_layers > NMR_MAX_LAYERS)
    return fail(NMR_ERR_ARG, std::string(what) + ": layer count out of range");
  if (!d->widths || !d->W || !d->b) return fail(NMR_ERR_ARG, std::string(what) + ": null arrays");
  for (int l = 0; l <= d->n_layers; ++l)
    if (d->widths[l] <= 0) return fail(NMR_ERR_ARG, std::string(what) + ": non-positive width");
  for (int l = 0; l < d->n_layers; ++l)
    if (!d->W[l] || !d->b[l]) return fail(NMR_ERR_ARG, std::string(what) + ": null layer");
  return NMR_OK;
}

// ---------------------------------------------------------------------------
// static scratch of cubature_force_stiffness_noalloc: every buffer beyond the
// caller's inputs and outputs (the instance table entry, the status word,
// the weighted element forces, the per-block partials and their sums) lives
// in one static device array.  Host code never passes the array's name to a
// kernel or a copy: its device address on each GPU comes from
// hipGetSymbolAddress at context creation (g_scratch_ptr).
static constexpr size_t kScratchBytes = (size_t)16 << 20;
static constexpr size_t kScratchHead = 4096;                  // Inst<T> table entry
static constexpr size_t kScratchStatus = kScratchHead;        // int status word
static constexpr size_t kScratchSums = kScratchHead + 256;    // [R*R + R] doubles
static constexpr size_t kScratchBody = kScratchSums + 8448;   // element forces, then partials
static_assert(sizeof(Inst<double>) <= kScratchHead && sizeof(Inst<float>) <= kScratchHead, "table entry size");
static_assert(NMR_MAX_R * NMR_MAX_R * 8 + NMR_MAX_R * 8 <= 8448 && kScratchBody % 256 == 0, "sums size");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

static constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// device address of `scratch` on the current device `device`, looked up once
static int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(NMR_ERR_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return NMR_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(NMR_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch_ptr[device] = p;
  return NMR_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int nmr_create(int device, void* hip_stream, size_t hbm_budget_bytes, nmr_ctx** out) {
  if (!out) return fail(NMR_ERR_ARG, "null out");
  *out = nullptr;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(NMR_ERR_ARG, "no such device");
  nmr_ctx* c = new nmr_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return fail(NMR_ERR_DEVICE, "hipSetDevice failed");
  }
  if (int rc = scratch_setup(device)) {
    delete c;
    return rc;
  }
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(NMR_ERR_DEVICE, "stream create failed");
    }
    c->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess) {
    delete c;
    return fail(NMR_ERR_DEVICE, "stream/event create failed");
  }
  *out = c;
  return NMR_OK;
}

extern "C" int nmr_destroy(nmr_ctx* c) {
  if (!c) return fail(NMR_ERR_ARG, "null ctx");
  CHK(set_device(c));
  (void)hipStreamSynchronize(c->stream);
  drop_many_graphs(c, nullptr);
  (void)hipStreamDestroy(c->cap);
  (void)hipEventDestroy(c->ev[0]);
  (void)hipEventDestroy(c->ev[1]);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return NMR_OK;
}

extern "C" const char* nmr_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// decoder
// ---------------------------------------------------------------------------
static int decoder_bytes(const nmr_mlp_desc* desc, int prec, size_t* bytes) {
  const int L = desc->n_layers;
  const size_t tw = prec == PREC_FP64 ? 8 : (prec == PREC_BF16 ? 2 : 4);
  const size_t tb = prec == PREC_FP64 ? 8 : 4;
  size_t b = 0;
  for (int l = 0; l < L; ++l) {
    const size_t ip = pad_to(desc->widths[l], NMR_WPAD), op = pad_to(desc->widths[l + 1], NMR_WPAD);
    b += round256(ip * op * tw) + round256(op * tb);
    if (l < L - 1) b += round256(ip * op * tw);
  }
  *bytes = b;
  return NMR_OK;
}

static int decoder_build(nmr_ctx* ctx, const nmr_mlp_desc* desc, int prec, nmr_decoder** out) {
  CHK(check_mlp(desc, 2, "decoder"));
  if (prec < PREC_FP64 || prec > PREC_BF16) return fail(NMR_ERR_ARG, "bad precision");
  if (desc->act < ACT_IDENTITY || desc->act > ACT_SIN) return fail(NMR_ERR_ARG, "bad activation");
  const int L = desc->n_layers;
  if (1 + desc->widths[0] > 64 || 4 + 4 * desc->widths[0] > 128)
    return fail(NMR_ERR_ARG, "decoder input size n_q must be <= 31");
  if (prec == PREC_FP64 && 4 + 4 * desc->widths[0] > 64)
    return fail(NMR_ERR_ARG, "FP64 decoders take n_q <= 15");
  if (prec != PREC_FP64 && pad_to(desc->widths[L - 1], NMR_WPAD) > 256)
    return fail(NMR_ERR_ARG, "the last hidden layer must be at most 256 wide");
  nmr_decoder* d = new nmr_decoder();
  d->ctx = ctx;
  d->d.L = L;
  d->d.act = desc->act;
  d->d.prec = prec;
  // the GEMM kernels take whole 32-wide K batches (the tall tiles' double
  // buffer, the BF16 K-steps), so every padded width is a multiple of 32
  static_assert(NMR_WPAD % 32 == 0, "layer widths must be padded to a multiple of 32");
  for (int l = 0; l <= L; ++l) {
    d->d.w[l] = desc->widths[l];
    d->d.wp[l] = pad_to(desc->widths[l], NMR_WPAD);
  }
  const size_t tw = prec == PREC_FP64 ? 8 : (prec == PREC_BF16 ? 2 : 4);
  const size_t tb = prec == PREC_FP64 ? 8 : 4;
  for (int l = 0; l < L; ++l) {
    const int in = d->d.w[l], outw = d->d.w[l + 1], ip = d->d.wp[l], op = d->d.wp[l + 1];
    std::vector<unsigned char> hw((size_t)ip * op * tw, 0), hb((size_t)op * tb, 0), ht;
    if (l < L - 1) ht.assign((size_t)ip * op * tw, 0);
    auto put = [&](std::vector<unsigned char>& v, size_t idx, double x) {
      if (prec == PREC_FP64) std::memcpy(&v[idx * 8], &x, 8);
      else if (prec == PREC_FP32) {
        float f = (float)x;
        std::memcpy(&v[idx * 4], &f, 4);
      } else {
        uint16_t h = f2bf((float)x);
        std::memcpy(&v[idx * 2], &h, 2);
      }
    };
    for (int o = 0; o < outw; ++o)
      for (int i = 0; i < in; ++i) {
        const double x = desc->W[l][(size_t)o * in + i];
        put(hw, (size_t)o * ip + i, x);
        if (l < L - 1) put(ht, (size_t)i * op + o, x);
      }
    for (int o = 0; o < outw; ++o) {
      const double x = desc->b[l][o];
      if (prec == PREC_FP64) std::memcpy(&hb[o * 8], &x, 8);
      else {
        float f = (float)x;
        std::memcpy(&hb[o * 4], &f, 4);
      }
    }
    void *pw, *pb, *pt = nullptr;
    int rc = dalloc(d->mem, hw.size(), &pw);
    if (rc == NMR_OK) rc = dalloc(d->mem, hb.size(), &pb);
    if (rc == NMR_OK && l < L - 1) rc = dalloc(d->mem, ht.size(), &pt);
    if (rc != NMR_OK) {
      d->mem.release();
      delete d;
      return rc;
    }
    if (hipMemcpy(pw, hw.data(), hw.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pb, hb.data(), hb.size(), hipMemcpyHostToDevice) != hipSuccess ||
        (pt && hipMemcpy(pt, ht.data(), ht.size(), hipMemcpyHostToDevice) != hipSuccess)) {
      d->mem.release();
      delete d;
      return fail(NMR_ERR_DEVICE, "decoder upload failed");
    }
    d->d.W[l] = pw;
    d->d.b[l] = pb;
    d->d.WT[l] = pt;
  }
  *out = d;
  return NMR_OK;
}

static void decoder_unref(nmr_decoder* d) {
  if (--d->refs == 0) {
    if (d->charged) d->ctx->used -= d->mem.bytes;
    d->ctx->used -= d->gram_mem.bytes;
    d->mem.release();
    d->gram_mem.release();
    delete d;
  }
}

// key of the output layer's Gram matrices: everything they depend on besides
// the decoder (FNV-1a over the mesh, pins, density, time step, gravity, the
// element type)
static uint64_t gram_key(const nmr_problem* p, int real_bytes) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* data, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  mix(&p->n_vertices, sizeof(int));
  mix(&p->n_tets, sizeof(int));
  mix(&real_bytes, sizeof(int));
  mix(&p->rho, sizeof(double));
  mix(&p->dt, sizeof(double));
  mix(p->gravity, 3 * sizeof(double));
  mix(p->X, (size_t)p->n_vertices * 3 * sizeof(double));
  mix(p->tets, (size_t)p->n_tets * 4 * sizeof(int32_t));
  mix(p->pinned, (size_t)p->n_vertices);
  return h;
}

extern "C" int nmr_decoder_create(nmr_ctx* ctx, const nmr_mlp_desc* desc, int prec, nmr_decoder** out) {
  if (!ctx || !out) return fail(NMR_ERR_ARG, "null argument");
  *out = nullptr;
  CHK(set_device(ctx));
  CHK(check_mlp(desc, 2, "decoder"));
  size_t bytes;
  decoder_bytes(desc, prec, &bytes);
  if (ctx->budget && ctx->used + bytes > ctx->budget) return fail(NMR_ERR_BUDGET, "decoder exceeds HBM budget");
  nmr_decoder* d;
  CHK(decoder_build(ctx, desc, prec, &d));
  d->charged = true;
  ctx->used += d->mem.bytes;
  *out = d;
  return NMR_OK;
}

extern "C" int nmr_decoder_destroy(nmr_decoder* d) {
  if (!d) return fail(NMR_ERR_ARG, "null decoder");
  CHK(set_device(d->ctx));
  (void)hipStreamSynchronize(d->ctx->stream);
  decoder_unref(d);
  return NMR_OK;
}

// ---------------------------------------------------------------------------
// instance
// ---------------------------------------------------------------------------
struct Sizes {
  int N, n, m, n_p, n_q, R, n_cub, L, Cp, Cb, Cf, Wmax, n_mblk, n_cblk, n_bblk, cub_per_blk;
  int wn_L, wn_maxw;
  int gram, K, n_cdofs, n_gblk, n_sblk, mblk_alloc, bblk_alloc;
  std::vector<int> cdofs;
};

template <typename T>
static size_t instance_bytes(const Sizes& s, const DecoderDev& d) {
  size_t b = 0;
  auto add = [&](size_t bytes) { b += round256(bytes); };
  const size_t t = sizeof(T);
  add(s.R * 8); add(s.R * 8); add(s.R * 8); add(3 * s.n_q * 8); add(kMaxIters * 8); add(4);
  add(s.N * t); add(s.N * t); add(s.N * t); add((size_t)s.N * s.n_p * t);
  add(s.n_cub * 16); add(s.n_cub * 9 * t); add(s.n_cub * t); add((s.n + 1) * 4); add(s.n_cub * 16);
  add(s.n_cub * t);
  add((size_t)s.Cp * s.Wmax * t); add((size_t)s.Cp * s.Wmax * t);
  for (int l = 0; l < s.L - 1; ++l) add((size_t)s.Cb * d.wp[l + 1] * t);
  add((size_t)s.Cf * d.wp[s.L - 1] * t);
  add((size_t)s.N * s.Cf * t); add(s.N * t);
  add((size_t)s.Cb * s.Wmax * t); add((size_t)s.Cb * s.Wmax * t);
  add((size_t)s.n_cub * 12 * t);
  add((size_t)s.n_cblk * (s.R * s.R + s.R) * 8);
  add((size_t)s.mblk_alloc * (s.R * s.R + s.R * s.n_q + s.R + s.n_p) * 8);
  add((size_t)s.bblk_alloc * d.wp[s.L - 1] * 8);
  if (s.gram) {
    add((size_t)s.n_cdofs * 4);
    add((size_t)s.K * s.K * 8);
    add((size_t)s.K * 8);
  }
  add((s.R * s.R + s.R) * 8); add((s.R * s.R + s.R * s.n_q + s.R + s.n_p) * 8);
  add(s.n_q * s.n_q * 8); add(s.n_q * 8);
  add((size_t)s.N * sizeof(T));  // frame
  if (s.n_p > 0) add((size_t)((s.N + 255) / 256) * s.n_p * s.Cf * 8);
  add(s.R * s.R * 8);
  return b;
}

template <typename T>
static int build_instance(nmr_ctx* ctx, const nmr_problem* p, int prec, nmr_decoder* dec, nmr_inst* in) {
  const DecoderDev& d = dec->d;
  Sizes s{};
  s.n = p->n_vertices;
  s.N = 3 * s.n;
  s.m = p->n_tets;
  s.n_p = p->n_p;
  s.n_q = d.w[0];
  s.R = s.n_p + s.n_q;
  s.n_cub = p->n_cub;
  s.L = d.L;
  // jet channels (complex steps) or stencil columns (central differences)
  const bool fd = p->fd_h > 0;
  s.Cp = fd ? pad_to(14 * s.n_q + 3, 16) : pad_to(4 + 4 * s.n_q, 16);
  s.Cb = fd ? pad_to(1 + 2 * s.n_q, 16) : pad_to(1 + s.n_q, 16);
  if (fd && s.Cp > (d.prec == PREC_FP64 ? 64 : 128))
    return fail(NMR_ERR_ARG, "central-difference derivatives need n_q <= 8 (n_q <= 4 in FP64)");
  s.Cf = pad_to(2 + 2 * s.n_q, 16);
  s.Wmax = 0;
  for (int l = 1; l < d.L; ++l) s.Wmax = std::max(s.Wmax, d.wp[l]);
  s.cub_per_blk = 4;  // four virtual waves of one tet (a 4-wave block, or four lane groups of one wave)
  s.n_mblk = (s.N + 255) / 256;
  s.n_cblk = (s.n_cub + s.cub_per_blk - 1) / s.cub_per_blk;
  s.n_bblk = (s.N + 127) / 128;
  // Gram-folded path: no linear subspace, last hidden layer <= 256
  s.K = d.wp[d.L - 1];
  s.gram = (p->newton_path == 0 && s.n_p == 0 && s.K <= 256) ? 1 : 0;
  s.n_cdofs = 0;
  s.n_gblk = kGramKParts * (s.K / 16);
  s.n_sblk = 0;
  if (s.gram) {
    std::vector<char> hit(s.N, 0);
    for (int c = 0; c < s.n_cub; ++c) {
      const int e = p->cub_ids[c];
      if (e < 0 || e >= p->n_tets) return fail(NMR_ERR_ARG, "cubature id out of range");
      for (int a = 0; a < 4; ++a) {
        const int v = p->tets[4 * e + a];
        if (v < 0 || v >= s.n) return fail(NMR_ERR_ARG, "tet vertex out of range");
        for (int k = 0; k < 3; ++k) hit[3 * v + k] = 1;
      }
    }
    for (int i = 0; i < s.N; ++i)
      if (hit[i]) s.cdofs.push_back(i);
    s.n_cdofs = (int)s.cdofs.size();
    s.n_sblk = (s.n_cdofs + 127) / 128;
  }
  s.mblk_alloc = std::max(s.n_mblk, s.n_gblk);
  s.bblk_alloc = std::max(s.n_bblk, s.n_sblk + kGramKParts);
  if (s.R > NMR_MAX_R - 1) return fail(NMR_ERR_ARG, "n_p + n_q must be <= 31");
  if (d.w[d.L] < s.N) return fail(NMR_ERR_ARG, "decoder output smaller than 3 * n_vertices");
  if (s.Cf > 64) return fail(NMR_ERR_ARG, "n_q too large for the output layer");
  s.wn_L = 0;
  s.wn_maxw = 0;
  if (!p->cub_w) {
    CHK(check_mlp(p->wnet, 1, "weight net"));
    if (p->wnet->widths[0] != s.R || p->wnet->widths[p->wnet->n_layers] != s.n_cub)
      return fail(NMR_ERR_ARG, "weight net must map R -> n_cub");
    s.wn_L = p->wnet->n_layers;
    for (int l = 0; l <= s.wn_L; ++l) s.wn_maxw = std::max(s.wn_maxw, p->wnet->widths[l]);
    for (int l = 0; l < s.wn_L; ++l)
      if (p->wnet->widths[l] > 1024) return fail(NMR_ERR_ARG, "weight-net hidden widths must be <= 1024");
  }
  size_t bytes = instance_bytes<T>(s, d);
  size_t wn_bytes = 0;
  if (s.wn_L)
    for (int l = 0; l < s.wn_L; ++l)
      wn_bytes += round256((size_t)p->wnet->widths[l] * p->wnet->widths[l + 1] * sizeof(T)) +
                  round256(p->wnet->widths[l + 1] * sizeof(T));
  bytes += wn_bytes + round256(2 * s.wn_maxw * sizeof(T)) + 2 * round256(sizeof(Inst<T>));
  if (!dec->charged) bytes += dec->mem.bytes;
  if (ctx->budget && ctx->used + bytes > ctx->budget) return fail(NMR_ERR_BUDGET, "instance exceeds HBM budget");

  in->N = s.N; in->n = s.n; in->n_p = s.n_p; in->n_q = s.n_q; in->R = s.R; in->n_cub = s.n_cub;
  in->Cp = s.Cp; in->Cb = s.Cb; in->Cf = s.Cf;
  in->n_mblk = s.n_mblk; in->n_cblk = s.n_cblk; in->n_bblk = s.n_bblk;
  in->gram = s.gram; in->n_cdofs = s.n_cdofs; in->n_sblk = s.n_sblk;
  in->cdofs = s.cdofs;
  in->fd = p->fd_h > 0 ? 1 : 0;
  in->m = s.m;
  in->Xh.assign(p->X, p->X + 3 * (size_t)s.n);
  in->tets_h.assign(p->tets, p->tets + 4 * (size_t)s.m);
  in->host.assign(sizeof(Inst<T>), 0);
  Inst<T>& I = host_inst<T>(in);
  I.active = 1;
  I.N = s.N; I.n = s.n; I.n_p = s.n_p; I.n_q = s.n_q; I.R = s.R; I.n_cub = s.n_cub;
  I.Cp = s.Cp; I.Cb = s.Cb; I.Cf = s.Cf; I.Np = pad_to(s.N, NMR_WPAD);
  I.n_mblk = s.n_mblk; I.n_cblk = s.n_cblk; I.n_bblk = s.n_bblk; I.cub_per_blk = s.cub_per_blk;
  I.dt = p->dt;
  I.mu = p->E / (2.0 * (1.0 + p->nu));
  I.lam = p->E * p->nu / ((1.0 + p->nu) * (1.0 - 2.0 * p->nu));
  for (int c = 0; c < 3; ++c) I.g[c] = p->gravity[c];

  DevMem& M = in->mem;
  CHK(dalloc_t(M, s.R, &I.r));
  CHK(dalloc_t(M, s.R, &I.rbar));
  CHK(dalloc_t(M, s.R, &I.rdot));
  CHK(dalloc_t(M, 3 * s.n_q, &I.dec_in));
  CHK(dalloc_t(M, kMaxIters, &I.resid));
  CHK(dalloc_t(M, 1, &I.status));
  T *X, *mass, *keep, *U = nullptr, *Bm, *Ve;
  int *cub_v, *csr_ptr, *csr_ent;
  CHK(dalloc_t(M, s.N, &X));
  CHK(dalloc_t(M, s.N, &mass));
  CHK(dalloc_t(M, s.N, &keep));
  CHK(dalloc_t(M, (size_t)s.N * s.n_p, &U));
  CHK(dalloc_t(M, 4 * s.n_cub, &cub_v));
  CHK(dalloc_t(M, 9 * s.n_cub, &Bm));
  CHK(dalloc_t(M, s.n_cub, &Ve));
  CHK(dalloc_t(M, s.n + 1, &csr_ptr));
  CHK(dalloc_t(M, 4 * s.n_cub, &csr_ent));
  CHK(dalloc_t(M, s.n_cub, &I.cub_w));
  I.X = X; I.mass = mass; I.keep = keep; I.U = U; I.cub_v = cub_v; I.cub_Bm = Bm; I.cub_Ve = Ve;
  I.csr_ptr = csr_ptr; I.csr_ent = csr_ent;
  CHK(dalloc_t(M, (size_t)s.Cp * s.Wmax, &I.act0));
  CHK(dalloc_t(M, (size_t)s.Cp * s.Wmax, &I.act1));
  for (int l = 0; l < s.L - 1; ++l) CHK(dalloc_t(M, (size_t)s.Cb * d.wp[l + 1], &I.pre[l]));
  CHK(dalloc_t(M, (size_t)s.Cf * d.wp[s.L - 1], &I.fold));
  CHK(dalloc_t(M, (size_t)s.N * s.Cf, &I.rec));
  CHK(dalloc_t(M, s.N, &I.seed));
  CHK(dalloc_t(M, (size_t)s.Cb * s.Wmax, &I.zb0));
  CHK(dalloc_t(M, (size_t)s.Cb * s.Wmax, &I.zb1));
  CHK(dalloc_t(M, (size_t)s.n_cub * 12, &I.fe));
  CHK(dalloc_t(M, (size_t)s.n_cblk * (s.R * s.R + s.R), &I.part_cub));
  CHK(dalloc_t(M, (size_t)s.mblk_alloc * (s.R * s.R + s.R * s.n_q + s.R + s.n_p), &I.part_mass));
  CHK(dalloc_t(M, (size_t)s.bblk_alloc * d.wp[s.L - 1], &I.part_bwd));
  I.gram = s.gram;
  I.trimmed = p->trimmed;
  I.fd = p->fd_h > 0 ? 1 : 0;
  I.fd_h = p->fd_h;
  I.n_gblk = s.n_gblk;
  I.n_cdofs = s.n_cdofs;
  I.n_sblk = s.n_sblk;
  bool gram_new = false;
  uint64_t gkey = 0;
  if (s.gram) {
    int* cd;
    CHK(dalloc_t(M, s.n_cdofs, &cd));
    HIPCHK(hipMemcpy(cd, s.cdofs.data(), s.n_cdofs * sizeof(int), hipMemcpyHostToDevice));
    I.cdofs = cd;
    gkey = gram_key(p, (int)sizeof(T));
    auto it = dec->gram_cache.find(gkey);
    if (it != dec->gram_cache.end()) {
      I.Gam = it->second.first;
      I.gam = it->second.second;
    } else {
      // computed below, after the lumped mass, and cached once that succeeded
      double *Gm, *gm;
      const size_t before = dec->gram_mem.bytes;
      CHK(dalloc_t(dec->gram_mem, (size_t)s.K * s.K, &Gm));
      CHK(dalloc_t(dec->gram_mem, s.K, &gm));
      ctx->used += dec->gram_mem.bytes - before;
      I.Gam = Gm;
      I.gam = gm;
      gram_new = true;
    }
  }
  CHK(dalloc_t(M, s.R * s.R + s.R, &I.sum_cub));
  CHK(dalloc_t(M, s.R * s.R + s.R * s.n_q + s.R + s.n_p, &I.sum_mass));
  CHK(dalloc_t(M, s.n_q * s.n_q, &I.Bq));
  CHK(dalloc_t(M, s.n_q, &I.JTa));
  CHK(dalloc_t(M, s.N, &I.frame));
  if (s.n_p > 0) CHK(dalloc_t(M, (size_t)((s.N + 255) / 256) * s.n_p * s.Cf, &I.part_filt));
  CHK(dalloc_t(M, s.R * s.R, &in->A_scratch));
  // cubature sources: the Newton path reads the decoder records
  I.cu_u = I.rec; I.cu_u_ld = s.Cf;
  I.cu_Ja = U; I.cu_Ja_ld = s.n_p; I.cu_na = s.n_p;
  I.cu_Jb = I.rec + 1; I.cu_Jb_ld = s.Cf; I.cu_nb = s.n_q;
  I.cu_w = I.cub_w;
  // weight net
  I.wn_L = s.wn_L;
  I.wn_scale = p->wnet_scale;
  I.wn_maxw = s.wn_maxw;
  for (int l = 0; l < s.wn_L; ++l) {
    const int wi = p->wnet->widths[l], wo = p->wnet->widths[l + 1];
    I.wn_w[l] = wi;
    I.wn_w[l + 1] = wo;
    std::vector<T> hw((size_t)wi * wo), hb(wo);
    for (size_t k = 0; k < hw.size(); ++k) hw[k] = (T)p->wnet->W[l][k];
    for (int o = 0; o < wo; ++o) hb[o] = (T)p->wnet->b[l][o];
    T *pw, *pb;
    CHK(dalloc_t(M, hw.size(), &pw));
    CHK(dalloc_t(M, hb.size(), &pb));
    HIPCHK(hipMemcpy(pw, hw.data(), hw.size() * sizeof(T), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(pb, hb.data(), hb.size() * sizeof(T), hipMemcpyHostToDevice));
    I.wn_W[l] = pw;
    I.wn_b[l] = pb;
  }
  if (s.wn_L) CHK(dalloc_t(M, 2 * (size_t)s.wn_maxw, &I.wn_buf));

  // host-side index bookkeeping and constant uploads
  {
    std::vector<T> hX(s.N), hkeep(s.N), hU((size_t)s.N * s.n_p);
    for (int i = 0; i < s.N; ++i) {
      hX[i] = (T)p->X[i];
      hkeep[i] = p->pinned[i / 3] ? T(0) : T(1);
    }
    for (size_t k = 0; k < hU.size(); ++k) hU[k] = (T)p->U[k];
    std::vector<int> hcv(4 * s.n_cub);
    for (int c = 0; c < s.n_cub; ++c) {
      const int e = p->cub_ids[c];
      if (e < 0 || e >= s.m) return fail(NMR_ERR_ARG, "cubature id out of range");
      for (int a = 0; a < 4; ++a) hcv[4 * c + a] = p->tets[4 * e + a];
    }
    for (int k = 0; k < 4 * s.m; ++k)
      if (p->tets[k] < 0 || p->tets[k] >= s.n) return fail(NMR_ERR_ARG, "tet vertex out of range");
    // vertex -> (cubature slot, corner), slots in increasing order
    std::vector<int> cnt(s.n + 1, 0), ent(4 * s.n_cub);
    for (int c = 0; c < s.n_cub; ++c)
      for (int a = 0; a < 4; ++a) cnt[hcv[4 * c + a] + 1]++;
    for (int v = 0; v < s.n; ++v) cnt[v + 1] += cnt[v];
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (int c = 0; c < s.n_cub; ++c)
      for (int a = 0; a < 4; ++a) ent[fill[hcv[4 * c + a]]++] = 4 * c + a;
    HIPCHK(hipMemcpy(X, hX.data(), s.N * sizeof(T), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(keep, hkeep.data(), s.N * sizeof(T), hipMemcpyHostToDevice));
    if (s.n_p) HIPCHK(hipMemcpy(U, hU.data(), hU.size() * sizeof(T), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(cub_v, hcv.data(), hcv.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(csr_ptr, cnt.data(), (s.n + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(csr_ent, ent.data(), ent.size() * 4, hipMemcpyHostToDevice));
    if (p->cub_w) {
      std::vector<T> hw(s.n_cub);
      for (int c = 0; c < s.n_cub; ++c) hw[c] = (T)p->cub_w[c];
      HIPCHK(hipMemcpy(I.cub_w, hw.data(), s.n_cub * sizeof(T), hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(I.rbar, p->r0, s.R * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(I.r, p->r0, s.R * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(I.rdot, p->rdot0, s.R * 8, hipMemcpyHostToDevice));
    // rest shape and lumped mass on the device (temporaries not charged)
    std::vector<int> vcnt(s.n + 1, 0), vent(4 * s.m);
    for (int e = 0; e < s.m; ++e)
      for (int a = 0; a < 4; ++a) vcnt[p->tets[4 * e + a] + 1]++;
    for (int v = 0; v < s.n; ++v) vcnt[v + 1] += vcnt[v];
    std::vector<int> vf(vcnt.begin(), vcnt.end() - 1);
    for (int e = 0; e < s.m; ++e)
      for (int a = 0; a < 4; ++a) vent[vf[p->tets[4 * e + a]]++] = e;
    DevMem tmp;
    double *dX, *dVe;
    int *dT, *dcub, *dvp, *dve;
    int rc = NMR_OK;
    if (rc == NMR_OK) rc = dalloc_t(tmp, s.N, &dX);
    if (rc == NMR_OK) rc = dalloc_t(tmp, s.m, &dVe);
    if (rc == NMR_OK) rc = dalloc_t(tmp, 4 * s.m, &dT);
    if (rc == NMR_OK) rc = dalloc_t(tmp, s.n_cub, &dcub);
    if (rc == NMR_OK) rc = dalloc_t(tmp, s.n + 1, &dvp);
    if (rc == NMR_OK) rc = dalloc_t(tmp, 4 * s.m, &dve);
    if (rc != NMR_OK) {
      tmp.release();
      return rc;
    }
    (void)hipMemcpy(dX, p->X, s.N * 8, hipMemcpyHostToDevice);
    (void)hipMemcpy(dT, p->tets, 16 * (size_t)s.m, hipMemcpyHostToDevice);
    (void)hipMemcpy(dcub, p->cub_ids, 4 * (size_t)s.n_cub, hipMemcpyHostToDevice);
    (void)hipMemcpy(dvp, vcnt.data(), 4 * (size_t)(s.n + 1), hipMemcpyHostToDevice);
    (void)hipMemcpy(dve, vent.data(), 4 * (size_t)(4 * s.m), hipMemcpyHostToDevice);
    launch_rest_shape<T>(dX, dT, s.m, dcub, s.n_cub, dvp, dve, s.n, p->rho, Bm, Ve, mass, dVe, ctx->stream);
    if (gram_new)
      launch_gram_setup<T>(d.W[d.L - 1], d.prec, s.K, mass, keep, s.N, p->dt, p->gravity, const_cast<double*>(I.Gam),
                           const_cast<double*>(I.gam), ctx->stream);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(ctx->stream);
    tmp.release();
    if (e1 != hipSuccess || e2 != hipSuccess) return fail(NMR_ERR_DEVICE, "rest-shape setup failed");
    if (gram_new) dec->gram_cache.emplace(gkey, std::make_pair(const_cast<double*>(I.Gam), const_cast<double*>(I.gam)));
  }
  // device copies of the instance table
  CHK(dalloc(M, sizeof(Inst<T>), &in->tab));
  CHK(dalloc(M, sizeof(Inst<T>), &in->api_tab));
  HIPCHK(hipMemcpy(in->tab, &I, sizeof(Inst<T>), hipMemcpyHostToDevice));
  in->bytes = M.bytes + (dec->charged ? 0 : dec->mem.bytes);
  return NMR_OK;
}

extern "C" int nmr_instance_create(nmr_ctx* ctx, const nmr_problem* p, int prec, nmr_inst** out) {
  if (!ctx || !p || !out) return fail(NMR_ERR_ARG, "null argument");
  *out = nullptr;
  CHK(set_device(ctx));
  if (prec < PREC_FP64 || prec > PREC_BF16) return fail(NMR_ERR_ARG, "bad precision");
  if (p->n_vertices <= 0 || !p->X || p->n_tets <= 0 || !p->tets || !p->pinned || p->n_cub <= 0 || !p->cub_ids ||
      !p->r0 || !p->rdot0 || p->n_p < 0 || (p->n_p > 0 && !p->U) || !(p->dt > 0) ||
      (p->trimmed != 0 && p->trimmed != 1) || !(p->fd_h >= 0) || !std::isfinite(p->fd_h))
    return fail(NMR_ERR_ARG, "incomplete problem");
  nmr_decoder* dec = p->shared_decoder;
  bool own = false;
  if (dec) {
    if (dec->ctx != ctx) return fail(NMR_ERR_ARG, "shared decoder belongs to another context");
    if (dec->d.prec != prec) return fail(NMR_ERR_ARG, "shared decoder precision differs");
  } else {
    size_t db;
    CHK(check_mlp(p->decoder, 2, "decoder"));
    decoder_bytes(p->decoder, prec, &db);
    if (ctx->budget && ctx->used + db > ctx->budget) return fail(NMR_ERR_BUDGET, "decoder exceeds HBM budget");
    CHK(decoder_build(ctx, p->decoder, prec, &dec));
    own = true;
  }
  nmr_inst* in = new nmr_inst();
  in->ctx = ctx;
  in->dec = dec;
  in->prec = prec;
  if (!own) dec->refs++;
  int rc = (prec == PREC_FP64) ? build_instance<double>(ctx, p, prec, dec, in)
                               : build_instance<float>(ctx, p, prec, dec, in);
  if (rc != NMR_OK) {
    std::string msg = g_err;
    in->mem.release();
    decoder_unref(dec);
    delete in;
    g_err = msg;
    return rc;
  }
  ctx->used += in->bytes;
  *out = in;
  return NMR_OK;
}

extern "C" int nmr_instance_destroy(nmr_inst* in) {
  if (!in) return fail(NMR_ERR_ARG, "null instance");
  nmr_ctx* c = in->ctx;
  CHK(set_device(c));
  (void)hipStreamSynchronize(c->stream);
  // an attached instance leaves its pool first: the pool's graph must never
  // reach the buffers freed below
  if (in->pool) CHK(nmr_pool_detach(in->pool, in->pool_slot));
  if (in->coupled_refs > 0) return fail(NMR_ERR_ARG, "instance is a member of a coupled set: destroy the set first");
  drop_many_graphs(c, in);
  for (auto& kv : in->step_graphs) (void)hipGraphExecDestroy(kv.second);
  c->used -= in->bytes;
  in->mem.release();
  decoder_unref(in->dec);
  delete in;
  return NMR_OK;
}

extern "C" int nmr_instance_bytes(const nmr_inst* in, size_t* bytes) {
  if (!in || !bytes) return fail(NMR_ERR_ARG, "null argument");
  *bytes = in->bytes;
  return NMR_OK;
}

extern "C" int nmr_instance_newton_path(const nmr_inst* in, int* path) {
  if (!in || !path) return fail(NMR_ERR_ARG, "null argument");
  *path = in->gram ? 0 : 1;
  return NMR_OK;
}

// ---------------------------------------------------------------------------
// launch sequences
// ---------------------------------------------------------------------------
struct Group {
  nmr_decoder* dec;
  bool f64;
  void* tab;  // device array of Inst<T>
  int nb, Cp, Cb, Cf, maxN, maxR, n_q, max_mblk, max_cblk, max_bblk, max_entries, max_cub;
  bool any_np;
  bool fd;  // central-difference derivatives (every member: the column count says so)
  bool gram;  // every table entry runs the Gram-folded path
  int max_cdofs, max_sblk, n_gblk, K;
  TileCfg tf[NMR_MAX_LAYERS], tb[NMR_MAX_LAYERS];  // hidden-layer tiles (ib == 0: the rule)
  bool same_rows;  // every member decodes the same output rows (checked exactly)
  const int* rows = nullptr;  // Gram path: the decoded rows every member shares (device), or null
  int n_rows = 0;
};

static Group group_of(const std::vector<nmr_inst*>& v, void* tab) {
  Group g{};
  g.dec = v[0]->dec;
  g.f64 = is_f64(v[0]);
  g.tab = tab;
  g.nb = (int)v.size();
  g.Cp = v[0]->Cp; g.Cb = v[0]->Cb; g.Cf = v[0]->Cf; g.n_q = v[0]->n_q;
  g.fd = v[0]->fd != 0;
  g.K = g.dec->d.wp[g.dec->d.L - 1];
  g.n_gblk = kGramKParts * (g.K / 16);
  g.gram = true;
  for (nmr_inst* in : v) {
    g.gram = g.gram && in->gram;
    g.max_cdofs = std::max(g.max_cdofs, in->n_cdofs);
    g.max_sblk = std::max(g.max_sblk, in->n_sblk);
    g.maxN = std::max(g.maxN, in->N);
    g.maxR = std::max(g.maxR, in->R);
    g.max_mblk = std::max(g.max_mblk, in->n_mblk);
    g.max_cblk = std::max(g.max_cblk, in->n_cblk);
    g.max_bblk = std::max(g.max_bblk, in->n_bblk);
    g.max_cub = std::max(g.max_cub, in->n_cub);
    g.max_entries = std::max(g.max_entries, 2 * in->R * in->R + in->R * in->n_q + 2 * in->R + in->n_p);
    g.any_np = g.any_np || in->n_p > 0;
  }
  g.same_rows = true;
  for (nmr_inst* in : v)
    g.same_rows = g.same_rows && (g.gram ? in->cdofs == v[0]->cdofs : in->N == v[0]->N);
  if (g.gram && g.same_rows) {
    g.rows = g.f64 ? host_inst<double>(v[0]).cdofs : host_inst<float>(v[0]).cdofs;
    g.n_rows = v[0]->n_cdofs;
  }
  return g;
}

// Channels the per-iteration output layer decodes into the records.  On the
// Gram-folded path the records feed only the cubature, which reads u and J:
// the value and the n_q J channels (the mass terms come from the folded
// activations).  The direct path decodes every channel.  The FP64 form
// always decodes every channel.
static int out_channels(const Group& g) {
  return (g.gram && !g.f64) ? pad_to(1 + g.n_q, 16) : g.Cf;
}

template <typename T>
static void enqueue_decoder_fwd(const Group& g, hipStream_t s, int add_up) {
  const DecoderDev& d = g.dec->d;
  const Inst<T>* tab = static_cast<const Inst<T>*>(g.tab);
  for (int l = 0; l < d.L - 1; ++l) launch_fwd_hidden<T>(d, l, tab, g.nb, g.Cp, g.fd, g.tf[l], s);
  launch_fwd_out<T>(d, tab, g.nb, g.gram ? g.max_cdofs : g.maxN, out_channels(g), g.same_rows, g.gram ? g.rows : nullptr,
                    s);
  if (g.any_np) launch_filter<T>(tab, g.nb, g.maxN, add_up, s);
}

// with_out: launch the output-layer backpropagation too (else the caller
// has, fused with the sums)
template <typename T>
static void enqueue_decoder_bwd(const Group& g, hipStream_t s, bool with_out = true) {
  const DecoderDev& d = g.dec->d;
  const Inst<T>* tab = static_cast<const Inst<T>*>(g.tab);
  if (with_out) {
    if (g.gram && g.rows && !g.f64 && g.nb >= 2) launch_bwd_out_batch<T>(d, tab, g.nb, g.rows, g.n_rows, s);
    else launch_bwd_out<T>(d, tab, g.nb, g.gram ? g.max_sblk : g.max_bblk, s);
  }
  launch_bwd_reduce<T>(d, tab, g.nb, s);
  for (int l = d.L - 2; l >= 0; --l) launch_bwd_hidden<T>(d, l, tab, g.nb, g.Cb, g.fd, g.tb[l], s);
}

// Independent kernels share a launch while the instances leave the chip
// idle; from this many instances on, each runs at its own occupancy (the
// shared grid takes the larger register and LDS footprint of the two).
static const int kShareLaunchMax = 16;
// frames of a Gram-path group as one GEMM over the instances from this many
static const int kFrameBatchMin = 8;

template <typename T>
static void enqueue_iteration(const Group& g, int iter, int mode, double* A_out, double* phi_out, hipStream_t s) {
  const Inst<T>* tab = static_cast<const Inst<T>*>(g.tab);
  enqueue_decoder_fwd<T>(g, s, 1);
  // a step's first iteration runs the decoder at r = rbar, the state the
  // step starts from: its value channel is that frame's displacement
  if (iter == 0 && (mode & SOLVE_UPDATE)) {
    if (g.gram && g.nb >= kFrameBatchMin) launch_frame_batch<T>(g.dec->d, tab, g.nb, g.maxN, s);
    else launch_frame<T>(g.dec->d, tab, g.nb, g.maxN, s);
  }
  if (g.gram && g.nb < kShareLaunchMax) {
    // the Gram terms need only the folded activations and the state, and the
    // output-layer seed only the element forces: each pair is one launch
    launch_cub_gram<T>(tab, g.nb, g.max_cblk, g.n_gblk, g.K, g.n_q, s);
    launch_sums_bwd_out<T>(g.dec->d, tab, g.nb, g.max_entries, g.max_sblk, g.max_cblk, s);
    enqueue_decoder_bwd<T>(g, s, false);
  } else {
    launch_cubature<T>(tab, g.nb, g.max_cblk, g.maxR, s);
    if (g.gram) launch_gram<T>(tab, g.nb, g.n_gblk, g.K, g.n_q, s);
    else launch_mass<T>(tab, g.nb, g.max_mblk, g.maxR, g.n_q, s);
    launch_sums<T>(tab, g.nb, g.max_entries, g.max_cblk, s);
    enqueue_decoder_bwd<T>(g, s);
  }
  launch_solve<T>(tab, g.nb, iter, mode, A_out, phi_out, s);
}

static void enqueue_step(const Group& g, int K, hipStream_t s) {
  for (int it = -1; it < K; ++it) {
    if (g.f64) {
      if (it < 0) launch_step_begin<double>(static_cast<const Inst<double>*>(g.tab), g.nb, BEGIN_STEP, g.max_cub, s);
      else enqueue_iteration<double>(g, it, SOLVE_UPDATE | (it == K - 1 ? SOLVE_FINISH : 0), nullptr, nullptr, s);
    } else {
      if (it < 0) launch_step_begin<float>(static_cast<const Inst<float>*>(g.tab), g.nb, BEGIN_STEP, g.max_cub, s);
      else enqueue_iteration<float>(g, it, SOLVE_UPDATE | (it == K - 1 ? SOLVE_FINISH : 0), nullptr, nullptr, s);
    }
  }
}

// ---------------------------------------------------------------------------
// tile choice of a group's hidden-layer launches
// ---------------------------------------------------------------------------
static const int kTuneReps = 10;

// Times every eligible configuration of one hidden layer on the group's own
// buffers (the layer only writes decoder scratch that the next real pass
// overwrites) and keeps the fastest for the context's lifetime.
template <typename T>
static int tune_layer(nmr_ctx* c, const Group& g, int l, bool fwd, TileCfg* out) {
  const DecoderDev& d = g.dec->d;
  const int cols = fwd ? g.Cp : g.Cb;
  const std::array<int, 7> key{fwd ? 1 : 0, d.wp[l], d.wp[l + 1], cols, g.nb, d.prec, g.fd ? 1 : 0};
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    *out = TileCfg{it->second.ib, it->second.mr, it->second.jet_groups};
    return NMR_OK;
  }
  TileCfg cand[8];
  const int n = tile_candidates(d, l, g.nb, cols, g.fd, g.f64, fwd, cand);
  *out = tile_rule(d, l, g.nb, cols, g.fd, g.f64, fwd);
  if (n <= 1) return NMR_OK;
  const Inst<T>* tab = static_cast<const Inst<T>*>(g.tab);
  float best = 0.f;
  for (int k = 0; k < n; ++k) {
    auto run = [&]() {
      if (fwd) launch_fwd_hidden<T>(d, l, tab, g.nb, g.Cp, g.fd, cand[k], c->stream);
      else launch_bwd_hidden<T>(d, l, tab, g.nb, g.Cb, g.fd, cand[k], c->stream);
    };
    run();
    run();
    HIPCHK(hipEventRecord(c->ev[0], c->stream));
    for (int r = 0; r < kTuneReps; ++r) run();
    HIPCHK(hipEventRecord(c->ev[1], c->stream));
    HIPCHK(hipEventSynchronize(c->ev[1]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    const float us = 1e3f * ms / kTuneReps;
    if (k == 0 || us < best) {
      best = us;
      *out = cand[k];
    }
  }
  HIPCHK(hipGetLastError());
  nmr_tile_choice e{key[0], key[1], key[2], key[3], key[4], key[5], out->ib, out->mr, out->jg, best};
  c->tuned.emplace(key, e);
  return NMR_OK;
}

// may_tune: the group's table holds live instances (timings mean something)
static int choose_tiles(nmr_ctx* c, Group& g, bool may_tune) {
  const DecoderDev& d = g.dec->d;
  for (int l = 0; l < d.L - 1; ++l)
    for (int fwd = 0; fwd < 2; ++fwd) {
      TileCfg& t = fwd ? g.tf[l] : g.tb[l];
      const int cols = fwd ? g.Cp : g.Cb;
      t = tile_rule(d, l, g.nb, cols, g.fd, g.f64, fwd);
      if (c->tile_mode == NMR_TILES_FORCE) {
        const TileCfg f{c->tile_ib, c->tile_mr};
        if (tile_eligible(d, l, g.nb, cols, g.fd, g.f64, fwd, f)) t = f;
      } else if (c->tile_mode == NMR_TILES_AUTOTUNE && may_tune) {
        CHK(g.f64 ? tune_layer<double>(c, g, l, fwd, &t) : tune_layer<float>(c, g, l, fwd, &t));
      }
    }
  return NMR_OK;
}

extern "C" int nmr_set_tiling(nmr_ctx* c, int mode, int ib, int mr) {
  if (!c) return fail(NMR_ERR_ARG, "null context");
  if (mode < NMR_TILES_RULE || mode > NMR_TILES_FORCE) return fail(NMR_ERR_ARG, "unknown tiling mode");
  if (mode == NMR_TILES_FORCE && !((ib == 1 || ib == 2 || ib == 4) && (mr == 1 || mr == 2 || mr == 4)))
    return fail(NMR_ERR_ARG, "forced tiles: ib and mr must be 1, 2 or 4");
  CHK(set_device(c));
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_many_graphs(c, nullptr);
  c->tile_mode = mode;
  c->tile_ib = mode == NMR_TILES_FORCE ? ib : 1;
  c->tile_mr = mode == NMR_TILES_FORCE ? mr : 1;
  c->tile_epoch++;
  return NMR_OK;
}

extern "C" int nmr_tiling_table(nmr_ctx* c, nmr_tile_choice* out, int cap, int* n) {
  if (!c || !n || cap < 0 || (cap > 0 && !out)) return fail(NMR_ERR_ARG, "bad argument");
  int k = 0;
  for (auto& kv : c->tuned) {
    if (k < cap) out[k] = kv.second;
    ++k;
  }
  *n = std::min(k, cap);
  return NMR_OK;
}

static int capture(nmr_ctx* c, const std::vector<Group>& groups, int K, hipGraphExec_t* exec) {
  hipGraph_t graph;
  HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
  for (const Group& g : groups) enqueue_step(g, K, c->cap);
  HIPCHK(hipStreamEndCapture(c->cap, &graph));
  hipError_t e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(NMR_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  return NMR_OK;
}

static int map_status(int st) {
  if (st & ST_INVERTED) return NMR_ERR_INVERTED;
  if (st & ST_NONFINITE) return NMR_ERR_NONFINITE;
  if (st & ST_SINGULAR) return NMR_ERR_SINGULAR;
  return NMR_OK;
}

static int read_status(nmr_inst* in, int* st) {
  const int* dst = is_f64(in) ? host_inst<double>(in).status : host_inst<float>(in).status;
  HIPCHK(hipStreamSynchronize(in->ctx->stream));
  HIPCHK(hipMemcpy(st, dst, sizeof(int), hipMemcpyDeviceToHost));
  return NMR_OK;
}

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
extern "C" int reduced_newton_step(nmr_inst* in, int n_iters, double* resid_norms_or_null) {
  if (!in) return fail(NMR_ERR_ARG, "null instance");
  if (n_iters < 1 || n_iters > kMaxIters) return fail(NMR_ERR_ARG, "n_iters must be in [1, 64]");
  nmr_ctx* c = in->ctx;
  CHK(set_device(c));
  auto it = in->step_graphs.find(n_iters);
  if (it == in->step_graphs.end()) {
    std::vector<nmr_inst*> v{in};
    hipGraphExec_t ex;
    CHK(capture(c, {group_of(v, in->tab)}, n_iters, &ex));
    it = in->step_graphs.emplace(n_iters, ex).first;
  }
  HIPCHK(hipGraphLaunch(it->second, c->stream));
  if (resid_norms_or_null) {
    const double* dres = is_f64(in) ? host_inst<double>(in).resid : host_inst<float>(in).resid;
    HIPCHK(hipMemcpyAsync(resid_norms_or_null, dres, n_iters * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    int st;
    CHK(read_status(in, &st));
    const int rc = map_status(st);
    if (rc != NMR_OK) return fail(rc, "instance failed during the step");
  }
  return NMR_OK;
}

extern "C" int step_many(nmr_ctx* c, nmr_inst* const* insts, int n_inst, int n_steps, int n_iters, int* status,
                         float* step_ms_or_null) {
  if (!c || !insts || n_inst <= 0 || n_steps < 0 || !status) return fail(NMR_ERR_ARG, "bad argument");
  if (n_iters < 1 || n_iters > kMaxIters) return fail(NMR_ERR_ARG, "n_iters must be in [1, 64]");
  CHK(set_device(c));
  std::vector<nmr_inst*> key(insts, insts + n_inst);
  for (nmr_inst* in : key)
    if (!in || in->ctx != c) return fail(NMR_ERR_ARG, "instance of another context");
  auto& per_k = c->many_graphs[key];
  auto git = per_k.find(n_iters);
  if (git == per_k.end()) {
    // group by decoder (instances sharing weights run as one batched launch)
    // and derivative scheme (the column count of the decoder passes)
    std::vector<std::pair<nmr_decoder*, std::vector<nmr_inst*>>> byd;
    for (nmr_inst* in : key) {
      auto f = std::find_if(byd.begin(), byd.end(),
                            [&](auto& pr) { return pr.first == in->dec && pr.second[0]->Cp == in->Cp; });
      if (f == byd.end()) byd.push_back({in->dec, {in}});
      else f->second.push_back(in);
    }
    GraphEntry ge;
    std::vector<Group> groups;
    for (auto& pr : byd) {
      const size_t isz = is_f64(pr.second[0]) ? sizeof(Inst<double>) : sizeof(Inst<float>);
      std::vector<unsigned char> host(isz * pr.second.size());
      bool all_gram = true;
      for (nmr_inst* x : pr.second) all_gram = all_gram && x->gram;
      for (size_t k = 0; k < pr.second.size(); ++k) {
        std::memcpy(&host[k * isz], pr.second[k]->host.data(), isz);
        // a group runs one path: the direct one unless every member can fold
        if (!all_gram) std::memset(&host[k * isz] + offsetof(Inst<float>, gram), 0, sizeof(int));
      }
      void* tab;
      HIPCHK(hipMalloc(&tab, host.size()));
      ge.tabs.push_back(tab);
      HIPCHK(hipMemcpy(tab, host.data(), host.size(), hipMemcpyHostToDevice));
      groups.push_back(group_of(pr.second, tab));
      int rc = choose_tiles(c, groups.back(), true);
      if (rc != NMR_OK) {
        for (void* p : ge.tabs) (void)hipFree(p);
        return rc;
      }
    }
    int rc = capture(c, groups, n_iters, &ge.exec);
    if (rc != NMR_OK) {
      for (void* p : ge.tabs) (void)hipFree(p);
      return rc;
    }
    git = per_k.emplace(n_iters, ge).first;
  }
  std::vector<hipEvent_t> ev;
  if (step_ms_or_null) {
    ev.resize(n_steps + 1);
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(ev[0], c->stream));
  }
  for (int s = 0; s < n_steps; ++s) {
    HIPCHK(hipGraphLaunch(git->second.exec, c->stream));
    if (step_ms_or_null) HIPCHK(hipEventRecord(ev[s + 1], c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  if (step_ms_or_null) {
    for (int s = 0; s < n_steps; ++s) HIPCHK(hipEventElapsedTime(&step_ms_or_null[s], ev[s], ev[s + 1]));
    for (auto& e : ev) (void)hipEventDestroy(e);
  }
  for (int k = 0; k < n_inst; ++k) {
    int st;
    CHK(read_status(key[k], &st));
    status[k] = map_status(st);
  }
  return NMR_OK;
}

// ---------------------------------------------------------------------------
// coupled sets: a core and rods tied to it (couple.hip), one graph per step
// ---------------------------------------------------------------------------
struct nmr_coupled {
  nmr_ctx* ctx = nullptr;
  std::vector<nmr_inst*> mem;  // core first
  bool f64 = false;
  DevMem dev;
  CoupleDev cd{};
  void* mem_tab = nullptr;
  std::vector<void*> group_tabs;
  std::vector<Group> groups;
  std::map<int, hipGraphExec_t> graphs;
  size_t bytes = 0;
};

template <typename T>
static int coupled_build(nmr_coupled* cs, const int32_t* ties, int n_tie) {
  nmr_ctx* c = cs->ctx;
  const int m = (int)cs->mem.size() - 1;
  const size_t isz = sizeof(Inst<T>);
  // per-member tie force and system buffers, then the member table and the
  // group tables (copies of the members' entries on the direct path)
  std::vector<Inst<T>> ent;
  for (nmr_inst* in : cs->mem) {
    Inst<T> I = host_inst<T>(in);
    CHK(dalloc_t(cs->dev, in->N, &I.pen));
    CHK(dalloc_t(cs->dev, (size_t)in->R * in->R, &I.sysA));
    CHK(dalloc_t(cs->dev, in->R, &I.sysphi));
    I.gram = 0;
    I.active = 1;
    ent.push_back(I);
  }
  CHK(dalloc(cs->dev, ent.size() * isz, &cs->mem_tab));
  HIPCHK(hipMemcpy(cs->mem_tab, ent.data(), ent.size() * isz, hipMemcpyHostToDevice));
  std::vector<std::pair<nmr_decoder*, std::vector<int>>> byd;
  for (int k = 0; k <= m; ++k) {
    nmr_inst* in = cs->mem[k];
    auto f = std::find_if(byd.begin(), byd.end(), [&](auto& pr) { return pr.first == in->dec; });
    if (f == byd.end()) byd.push_back({in->dec, {k}});
    else f->second.push_back(k);
  }
  for (auto& pr : byd) {
    std::vector<Inst<T>> ge;
    std::vector<nmr_inst*> v;
    for (int k : pr.second) {
      ge.push_back(ent[k]);
      v.push_back(cs->mem[k]);
    }
    void* tab;
    CHK(dalloc(cs->dev, ge.size() * isz, &tab));
    HIPCHK(hipMemcpy(tab, ge.data(), ge.size() * isz, hipMemcpyHostToDevice));
    cs->group_tabs.push_back(tab);
    Group g = group_of(v, tab);
    g.gram = false;
    g.same_rows = false;
    CHK(choose_tiles(c, g, false));
    cs->groups.push_back(g);
  }
  // ties: DOF pairs (rod DOF, core DOF) per rod
  const int ntd = 3 * n_tie;
  std::vector<int> td((size_t)m * ntd * 2);
  for (int k = 0; k < m; ++k)
    for (int t = 0; t < n_tie; ++t)
      for (int d = 0; d < 3; ++d) {
        const size_t o = 2 * ((size_t)k * ntd + 3 * t + d);
        td[o] = 3 * ties[2 * ((size_t)k * n_tie + t)] + d;
        td[o + 1] = 3 * ties[2 * ((size_t)k * n_tie + t) + 1] + d;
      }
  int* dtie;
  CHK(dalloc_t(cs->dev, td.size(), &dtie));
  HIPCHK(hipMemcpy(dtie, td.data(), td.size() * sizeof(int), hipMemcpyHostToDevice));
  cs->cd.n_rods = m;
  cs->cd.n_td = ntd;
  cs->cd.tie = dtie;
  CHK(dalloc_t(cs->dev, (size_t)m * kCoupleWs, &cs->cd.ws));
  CHK(dalloc_t(cs->dev, NMR_MAX_R, &cs->cd.dc));
  CHK(dalloc_t(cs->dev, NMR_MAX_R * NMR_MAX_R + 2 * NMR_MAX_R + 1, &cs->cd.red));
  CHK(dalloc_t(cs->dev, 1, &cs->cd.frozen));
  return NMR_OK;
}

template <typename T>
static void enqueue_coupled_step(nmr_coupled* cs, int K, hipStream_t s) {
  const Inst<T>* mt = static_cast<const Inst<T>*>(cs->mem_tab);
  for (const Group& g : cs->groups)
    launch_step_begin<T>(static_cast<const Inst<T>*>(g.tab), g.nb, BEGIN_STEP, g.max_cub, s);
  for (int it = 0; it < K; ++it) {
    const int mode = SOLVE_UPDATE | (it == K - 1 ? SOLVE_FINISH : 0);
    for (const Group& g : cs->groups) {
      enqueue_decoder_fwd<T>(g, s, 1);
      if (it == 0) launch_frame<T>(g.dec->d, static_cast<const Inst<T>*>(g.tab), g.nb, g.maxN, s);
    }
    launch_couple_pen<T>(mt, cs->cd, s);
    for (const Group& g : cs->groups) {
      const Inst<T>* tab = static_cast<const Inst<T>*>(g.tab);
      launch_cubature<T>(tab, g.nb, g.max_cblk, g.maxR, s);
      launch_mass<T>(tab, g.nb, g.max_mblk, g.maxR, g.n_q, s);
      launch_sums<T>(tab, g.nb, g.max_entries, g.max_cblk, s);
      enqueue_decoder_bwd<T>(g, s);
      launch_solve<T>(tab, g.nb, it, SOLVE_WRITE_SYSTEM | SOLVE_WRITE_INST, nullptr, nullptr, s);
    }
    launch_couple_solve<T>(mt, cs->cd, it, mode, s);
  }
}

extern "C" int nmr_coupled_create(nmr_ctx* c, nmr_inst* core, int n_rods, nmr_inst* const* rods,
                                  const int32_t* ties, int n_tie, double kappa, nmr_coupled** out) {
  if (!c || !core || n_rods < 1 || !rods || !ties || n_tie < 1 || !out) return fail(NMR_ERR_ARG, "bad argument");
  if (!(kappa >= 0.0) || !std::isfinite(kappa)) return fail(NMR_ERR_ARG, "kappa must be finite and >= 0");
  if (3 * n_tie > 64) return fail(NMR_ERR_ARG, "at most 21 tied vertices per rod");
  *out = nullptr;
  CHK(set_device(c));
  std::vector<nmr_inst*> mem{core};
  for (int k = 0; k < n_rods; ++k) mem.push_back(rods[k]);
  for (nmr_inst* in : mem) {
    if (!in || in->ctx != c) return fail(NMR_ERR_ARG, "instance of another context");
    if (in->prec != core->prec) return fail(NMR_ERR_ARG, "members must share one precision");
    if (in->fd) return fail(NMR_ERR_ARG, "coupled members take complex-step derivatives");
    if (in->pool) return fail(NMR_ERR_ARG, "a member is attached to a pool");
    auto dt_of = [](nmr_inst* x) { return is_f64(x) ? host_inst<double>(x).dt : host_inst<float>(x).dt; };
    if (dt_of(in) != dt_of(core)) return fail(NMR_ERR_ARG, "members must share the time step");
  }
  for (size_t a = 0; a < mem.size(); ++a)
    for (size_t b = a + 1; b < mem.size(); ++b)
      if (mem[a] == mem[b]) return fail(NMR_ERR_ARG, "an instance appears twice");
  std::vector<char> used(core->N, 0);
  for (int k = 0; k < n_rods; ++k)
    for (int t = 0; t < n_tie; ++t) {
      const int vr = ties[2 * ((size_t)k * n_tie + t)], vc = ties[2 * ((size_t)k * n_tie + t) + 1];
      if (vr < 0 || 3 * vr >= rods[k]->N || vc < 0 || 3 * vc >= core->N) return fail(NMR_ERR_ARG, "tie vertex out of range");
      if (used[3 * vc]) return fail(NMR_ERR_ARG, "a core vertex is tied twice");
      used[3 * vc] = 1;
    }
  nmr_coupled* cs = new nmr_coupled();
  cs->ctx = c;
  cs->mem = mem;
  cs->f64 = is_f64(core);
  cs->cd.kappa = kappa;
  int rc = cs->f64 ? coupled_build<double>(cs, ties, n_tie) : coupled_build<float>(cs, ties, n_tie);
  if (rc == NMR_OK && c->budget && c->used + cs->dev.bytes > c->budget) rc = fail(NMR_ERR_BUDGET, "coupled set exceeds HBM budget");
  if (rc != NMR_OK) {
    cs->dev.release();
    delete cs;
    return rc;
  }
  c->used += cs->dev.bytes;
  for (nmr_inst* in : mem) in->coupled_refs++;
  *out = cs;
  return NMR_OK;
}

extern "C" int nmr_coupled_destroy(nmr_coupled* cs) {
  if (!cs) return fail(NMR_ERR_ARG, "null coupled set");
  CHK(set_device(cs->ctx));
  (void)hipStreamSynchronize(cs->ctx->stream);
  for (auto& kv : cs->graphs) (void)hipGraphExecDestroy(kv.second);
  cs->ctx->used -= cs->dev.bytes;
  cs->dev.release();
  for (nmr_inst* in : cs->mem) in->coupled_refs--;
  delete cs;
  return NMR_OK;
}

extern "C" int nmr_coupled_step(nmr_coupled* cs, int n_steps, int n_iters, int* status, float* step_ms_or_null) {
  if (!cs || n_steps < 0 || !status) return fail(NMR_ERR_ARG, "bad argument");
  if (n_iters < 1 || n_iters > kMaxIters) return fail(NMR_ERR_ARG, "n_iters must be in [1, 64]");
  nmr_ctx* c = cs->ctx;
  CHK(set_device(c));
  auto it = cs->graphs.find(n_iters);
  if (it == cs->graphs.end()) {
    hipGraph_t graph;
    HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
    if (cs->f64) enqueue_coupled_step<double>(cs, n_iters, c->cap);
    else enqueue_coupled_step<float>(cs, n_iters, c->cap);
    HIPCHK(hipStreamEndCapture(c->cap, &graph));
    hipGraphExec_t ex;
    hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(NMR_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    it = cs->graphs.emplace(n_iters, ex).first;
  }
  std::vector<hipEvent_t> ev;
  if (step_ms_or_null) {
    ev.resize(n_steps + 1);
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(ev[0], c->stream));
  }
  for (int s = 0; s < n_steps; ++s) {
    HIPCHK(hipGraphLaunch(it->second, c->stream));
    if (step_ms_or_null) HIPCHK(hipEventRecord(ev[s + 1], c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  if (step_ms_or_null) {
    for (int s = 0; s < n_steps; ++s) HIPCHK(hipEventElapsedTime(&step_ms_or_null[s], ev[s], ev[s + 1]));
    for (auto& e : ev) (void)hipEventDestroy(e);
  }
  for (size_t k = 0; k < cs->mem.size(); ++k) {
    int st;
    CHK(read_status(cs->mem[k], &st));
    status[k] = map_status(st);
  }
  return NMR_OK;
}

// the instance table with the direct (all-DOF) output layer, in the scratch
// slot: used by the calls that return full-space arrays
template <typename T>
static int direct_tab(nmr_inst* in, void** out) {
  Inst<T> I = host_inst<T>(in);
  I.gram = 0;
  HIPCHK(hipStreamSynchronize(in->ctx->stream));
  HIPCHK(hipMemcpy(in->api_tab, &I, sizeof(Inst<T>), hipMemcpyHostToDevice));
  *out = in->api_tab;
  return NMR_OK;
}

template <typename T>
static int djh_impl(nmr_inst* in, const double* q, const double* dq, const double* qdot, const void* a, void* u,
                    void* J, void* dJ, void* Hdd, double* B, double* JTa) {
  nmr_ctx* c = in->ctx;
  Inst<T>& I = host_inst<T>(in);
  const size_t nqb = in->n_q * sizeof(double);
  HIPCHK(hipMemcpyAsync(I.dec_in, q, nqb, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(I.dec_in + in->n_q, dq, nqb, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(I.dec_in + 2 * in->n_q, qdot, nqb, hipMemcpyDeviceToDevice, c->stream));
  void* dt_tab;
  CHK(direct_tab<T>(in, &dt_tab));
  const Inst<T>* tab = static_cast<const Inst<T>*>(dt_tab);
  std::vector<nmr_inst*> v{in};
  Group g = group_of(v, dt_tab);
  g.gram = false;
  enqueue_decoder_fwd<T>(g, c->stream, 0);
  launch_unpack<T>(tab, (T*)u, (T*)J, (T*)dJ, (T*)Hdd, in->N, c->stream);
  if (a) {
    launch_seed_from_a<T>(tab, static_cast<const T*>(a), 1, in->n_mblk, c->stream);
    launch_sums<T>(tab, 1, g.max_entries, g.max_cblk, c->stream);
    enqueue_decoder_bwd<T>(g, c->stream);
    if (B) HIPCHK(hipMemcpyAsync(B, I.Bq, in->n_q * nqb, hipMemcpyDeviceToDevice, c->stream));
    if (JTa) HIPCHK(hipMemcpyAsync(JTa, I.JTa, nqb, hipMemcpyDeviceToDevice, c->stream));
  }
  HIPCHK(hipGetLastError());
  return NMR_OK;
}

extern "C" int decoder_jacobian_hessian(nmr_inst* in, const double* q, const double* dq, const double* qdot_bar,
                                        const void* a_or_null, void* u, void* J, void* dJ, void* Hdd,
                                        double* B_or_null, double* JTa_or_null) {
  if (!in || !q || !dq || !qdot_bar || !u || !J || !dJ || !Hdd) return fail(NMR_ERR_ARG, "null argument");
  CHK(set_device(in->ctx));
  return is_f64(in) ? djh_impl<double>(in, q, dq, qdot_bar, a_or_null, u, J, dJ, Hdd, B_or_null, JTa_or_null)
                    : djh_impl<float>(in, q, dq, qdot_bar, a_or_null, u, J, dJ, Hdd, B_or_null, JTa_or_null);
}

template <typename T>
static int cfs_impl(nmr_inst* in, const void* u, const void* Jt, const void* w, void* f_int, double* fr, double* Kr) {
  nmr_ctx* c = in->ctx;
  int st0;
  CHK(read_status(in, &st0));
  Inst<T> I = host_inst<T>(in);
  I.cu_u = static_cast<const T*>(u);
  I.cu_u_ld = 1;
  I.cu_Ja = static_cast<const T*>(Jt);
  I.cu_Ja_ld = in->R;
  I.cu_na = in->R;
  I.cu_Jb = nullptr;
  I.cu_Jb_ld = 0;
  I.cu_nb = 0;
  if (w) I.cu_w = static_cast<const T*>(w);
  I.gram = 0;
  HIPCHK(hipMemcpy(in->api_tab, &I, sizeof(Inst<T>), hipMemcpyHostToDevice));
  const Inst<T>* tab = static_cast<const Inst<T>*>(in->api_tab);
  launch_cubature<T>(tab, 1, in->n_cblk, in->R, c->stream);
  std::vector<nmr_inst*> v{in};
  Group g = group_of(v, in->api_tab);
  launch_sums<T>(tab, 1, g.max_entries, g.max_cblk, c->stream);
  HIPCHK(hipMemcpyAsync(Kr, I.sum_cub, in->R * in->R * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(fr, I.sum_cub + in->R * in->R, in->R * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (f_int) launch_fint<T>(tab, static_cast<T*>(f_int), in->N, c->stream);
  HIPCHK(hipGetLastError());
  int st;
  CHK(read_status(in, &st));
  if ((st & ST_INVERTED) && !(st0 & ST_INVERTED)) {
    HIPCHK(hipMemcpy(I.status, &st0, sizeof(int), hipMemcpyHostToDevice));
    return fail(NMR_ERR_INVERTED, "a cubature tet has det F <= 0");
  }
  return NMR_OK;
}

extern "C" int cubature_force_stiffness(nmr_inst* in, const void* u, const void* Jt, const void* w_or_null,
                                        void* f_int_or_null, double* fr, double* Kr) {
  if (!in || !u || !Jt || !fr || !Kr) return fail(NMR_ERR_ARG, "null argument");
  CHK(set_device(in->ctx));
  return is_f64(in) ? cfs_impl<double>(in, u, Jt, w_or_null, f_int_or_null, fr, Kr)
                    : cfs_impl<float>(in, u, Jt, w_or_null, f_int_or_null, fr, Kr);
}

// ---------------------------------------------------------------------------
// cubature_force_stiffness_noalloc: the kernels of cubature_force_stiffness
// on the static scratch
// ---------------------------------------------------------------------------
// bytes of the static scratch that cubature_force_stiffness_noalloc needs
template <typename T>
static size_t noalloc_bytes(const nmr_inst* in) {
  const size_t fe = round256((size_t)in->n_cub * 12 * sizeof(T));
  const size_t part = (size_t)in->n_cblk * (in->R * in->R + in->R) * sizeof(double);
  return kScratchBody + fe + part;
}

template <typename T>
static int cfs_noalloc_impl(nmr_inst* in, const void* u, const void* Jt, const void* w, void* f_int, double* fr,
                            double* Kr) {
  nmr_ctx* c = in->ctx;
  const size_t need = noalloc_bytes<T>(in);
  if (need > kScratchBytes)
    return fail(NMR_ERR_ARG, "cubature set too large for the static scratch: needs " + std::to_string(need) +
                                 " bytes, the limit is " + std::to_string(kScratchBytes));
  unsigned char* base = static_cast<unsigned char*>(g_scratch_ptr[c->device]);
  if (!base) return fail(NMR_ERR_DEVICE, "scratch address not set up for this device");
  // the table entry and a zero status word, written in one copy
  struct Head {
    Inst<T> I;
    unsigned char pad[kScratchStatus - sizeof(Inst<T>)];
    int status;
  } head;
  static_assert(offsetof(Head, status) == kScratchStatus, "status offset");
  std::memset(&head, 0, sizeof(head));
  head.I = host_inst<T>(in);
  Inst<T>& I = head.I;
  I.cu_u = static_cast<const T*>(u);
  I.cu_u_ld = 1;
  I.cu_Ja = static_cast<const T*>(Jt);
  I.cu_Ja_ld = in->R;
  I.cu_na = in->R;
  I.cu_Jb = nullptr;
  I.cu_Jb_ld = 0;
  I.cu_nb = 0;
  if (w) I.cu_w = static_cast<const T*>(w);
  I.gram = 0;
  I.status = reinterpret_cast<int*>(base + kScratchStatus);
  I.sum_cub = reinterpret_cast<double*>(base + kScratchSums);
  I.fe = reinterpret_cast<T*>(base + kScratchBody);
  I.part_cub = reinterpret_cast<double*>(base + kScratchBody + round256((size_t)in->n_cub * 12 * sizeof(T)));
  head.status = 0;
  // earlier work on the stream may still read the scratch (an earlier call)
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(base, &head, sizeof(head), hipMemcpyHostToDevice));
  const Inst<T>* tab = reinterpret_cast<const Inst<T>*>(base);
  launch_cubature<T>(tab, 1, in->n_cblk, in->R, c->stream);
  const int Ec = in->R * in->R + in->R;
  launch_sums<T>(tab, 1, Ec, in->n_cblk, c->stream);  // cubature entries only
  HIPCHK(hipMemcpyAsync(Kr, I.sum_cub, in->R * in->R * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(fr, I.sum_cub + in->R * in->R, in->R * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (f_int) launch_fint<T>(tab, static_cast<T*>(f_int), in->N, c->stream);
  HIPCHK(hipGetLastError());
  int st = 0;
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(&st, I.status, sizeof(int), hipMemcpyDeviceToHost));
  if (st & ST_INVERTED) return fail(NMR_ERR_INVERTED, "a cubature tet has det F <= 0");
  return NMR_OK;
}

extern "C" int cubature_force_stiffness_noalloc(nmr_inst* in, const void* u, const void* Jt, const void* w_or_null,
                                                void* f_int_or_null, double* fr, double* Kr) {
  if (!in || !u || !Jt || !fr || !Kr) return fail(NMR_ERR_ARG, "null argument");
  CHK(set_device(in->ctx));
  return is_f64(in) ? cfs_noalloc_impl<double>(in, u, Jt, w_or_null, f_int_or_null, fr, Kr)
                    : cfs_noalloc_impl<float>(in, u, Jt, w_or_null, f_int_or_null, fr, Kr);
}

template <typename T>
static int sys_impl(nmr_inst* in, const double* r, double* A, double* phi) {
  nmr_ctx* c = in->ctx;
  Inst<T>& I = host_inst<T>(in);
  HIPCHK(hipMemcpyAsync(I.r, r, in->R * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  std::vector<nmr_inst*> v{in};
  Group g = group_of(v, in->tab);
  launch_step_begin<T>(static_cast<const Inst<T>*>(in->tab), 1, BEGIN_SYSTEM, in->n_cub, c->stream);
  enqueue_iteration<T>(g, 0, SOLVE_WRITE_SYSTEM, A, phi, c->stream);
  HIPCHK(hipGetLastError());
  return NMR_OK;
}

extern "C" int reduced_newton_system(nmr_inst* in, const double* r, double* A, double* phi) {
  if (!in || !r || !A || !phi) return fail(NMR_ERR_ARG, "null argument");
  CHK(set_device(in->ctx));
  return is_f64(in) ? sys_impl<double>(in, r, A, phi) : sys_impl<float>(in, r, A, phi);
}

template <typename T>
static int get_state_impl(nmr_inst* in, double* r, double* rdot, void* u) {
  nmr_ctx* c = in->ctx;
  Inst<T>& I = host_inst<T>(in);
  HIPCHK(hipStreamSynchronize(c->stream));
  if (r) HIPCHK(hipMemcpy(r, I.rbar, in->R * sizeof(double), hipMemcpyDeviceToHost));
  if (rdot) HIPCHK(hipMemcpy(rdot, I.rdot, in->R * sizeof(double), hipMemcpyDeviceToHost));
  if (u) {
    // decode the frame at rbar: r <- rbar, decoder input (qbar, 0, rdot_bar),
    // the instance's own forward pass, then u = U p + D(q) into its frame buffer
    HIPCHK(hipMemcpyAsync(I.r, I.rbar, in->R * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    const Inst<T>* tab = static_cast<const Inst<T>*>(in->tab);
    launch_step_begin<T>(tab, 1, BEGIN_SYSTEM, in->n_cub, c->stream);
    std::vector<nmr_inst*> v{in};
    Group g = group_of(v, in->tab);
    enqueue_decoder_fwd<T>(g, c->stream, 1);
    launch_frame<T>(g.dec->d, tab, 1, in->N, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(u, I.frame, in->N * sizeof(T), hipMemcpyDeviceToHost));
  }
  return NMR_OK;
}

template <typename T>
static int get_frame_impl(nmr_inst* in, void* u) {
  HIPCHK(hipStreamSynchronize(in->ctx->stream));
  HIPCHK(hipMemcpy(u, host_inst<T>(in).frame, in->N * sizeof(T), hipMemcpyDeviceToHost));
  return NMR_OK;
}

extern "C" int nmr_instance_get_frame(nmr_inst* in, void* u) {
  if (!in || !u) return fail(NMR_ERR_ARG, "null argument");
  CHK(set_device(in->ctx));
  return is_f64(in) ? get_frame_impl<double>(in, u) : get_frame_impl<float>(in, u);
}

extern "C" int nmr_instance_frame_ptr(nmr_inst* in, void** u_dev) {
  if (!in || !u_dev) return fail(NMR_ERR_ARG, "null argument");
  *u_dev = is_f64(in) ? (void*)host_inst<double>(in).frame : (void*)host_inst<float>(in).frame;
  return NMR_OK;
}

extern "C" int nmr_instance_get_state(nmr_inst* in, double* r, double* rdot, void* u_or_null) {
  if (!in) return fail(NMR_ERR_ARG, "null instance");
  CHK(set_device(in->ctx));
  return is_f64(in) ? get_state_impl<double>(in, r, rdot, u_or_null) : get_state_impl<float>(in, r, rdot, u_or_null);
}

extern "C" int nmr_instance_set_state(nmr_inst* in, const double* r, const double* rdot) {
  if (!in || !r || !rdot) return fail(NMR_ERR_ARG, "null argument");
  CHK(set_device(in->ctx));
  double *rb, *rd;
  int* st;
  if (is_f64(in)) {
    rb = host_inst<double>(in).rbar; rd = host_inst<double>(in).rdot; st = host_inst<double>(in).status;
  } else {
    rb = host_inst<float>(in).rbar; rd = host_inst<float>(in).rdot; st = host_inst<float>(in).status;
  }
  HIPCHK(hipStreamSynchronize(in->ctx->stream));
  HIPCHK(hipMemcpy(rb, r, in->R * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(rd, rdot, in->R * sizeof(double), hipMemcpyHostToDevice));
  const int zero = 0;
  HIPCHK(hipMemcpy(st, &zero, sizeof(int), hipMemcpyHostToDevice));
  return NMR_OK;
}

// ---------------------------------------------------------------------------
// slot pools: one graph over `capacity` table entries; attach / detach rewrite
// one entry of the device table between steps
// ---------------------------------------------------------------------------
struct nmr_pool {
  nmr_ctx* ctx = nullptr;
  int capacity = 0;
  std::vector<nmr_inst*> slots;
  nmr_inst proto_copy;        // class representative (sizes, decoder), a copy
  nmr_inst* proto = nullptr;  // &proto_copy once the first instance attached
  void* tab = nullptr;        // device table of capacity Inst<T>
  size_t isz = 0;
  std::map<int, hipGraphExec_t> graphs;
  int tile_epoch = 0;  // the context's tiling epoch the graphs were captured in
  int* rows = nullptr;  // Gram path: the class's decoded rows (device copy; every member shares them)
};

extern "C" int nmr_pool_create(nmr_ctx* c, int capacity, nmr_pool** out) {
  if (!c || !out || capacity < 1) return fail(NMR_ERR_ARG, "bad argument");
  CHK(set_device(c));
  nmr_pool* p = new nmr_pool();
  p->ctx = c;
  p->capacity = capacity;
  p->slots.assign(capacity, nullptr);
  *out = p;
  return NMR_OK;
}

static void pool_drop_graphs(nmr_pool* p) {
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  p->graphs.clear();
}

extern "C" int nmr_pool_destroy(nmr_pool* p) {
  if (!p) return fail(NMR_ERR_ARG, "null pool");
  CHK(set_device(p->ctx));
  (void)hipStreamSynchronize(p->ctx->stream);
  for (nmr_inst* x : p->slots)
    if (x) {
      x->pool = nullptr;
      x->pool_slot = -1;
    }
  pool_drop_graphs(p);
  if (p->tab) (void)hipFree(p->tab);
  if (p->rows) (void)hipFree(p->rows);
  if (p->proto) decoder_unref(p->proto->dec);
  delete p;
  return NMR_OK;
}

// The pool's graph is captured from its first instance: its launch grids,
// its Newton path (Gram-folded or direct), the decoded rows of the Gram path,
// the formulation, the derivative scheme and the weight net's shape must
// hold for every later member too.
template <typename T>
static bool same_inst_shape(const nmr_inst* a, const nmr_inst* b) {
  const Inst<T>& x = *reinterpret_cast<const Inst<T>*>(a->host.data());
  const Inst<T>& y = *reinterpret_cast<const Inst<T>*>(b->host.data());
  if (x.trimmed != y.trimmed || x.fd != y.fd || x.fd_h != y.fd_h || x.wn_L != y.wn_L || x.wn_maxw != y.wn_maxw)
    return false;
  for (int l = 0; x.wn_L > 0 && l <= x.wn_L; ++l)
    if (x.wn_w[l] != y.wn_w[l]) return false;
  return true;
}

static bool same_class(const nmr_inst* a, const nmr_inst* b) {
  if (!(a->dec == b->dec && a->prec == b->prec && a->Cp == b->Cp && a->Cb == b->Cb && a->Cf == b->Cf &&
        a->N == b->N && a->n_p == b->n_p && a->n_q == b->n_q && a->n_cub == b->n_cub && a->n_mblk == b->n_mblk &&
        a->n_cblk == b->n_cblk && a->n_bblk == b->n_bblk && a->gram == b->gram && a->n_cdofs == b->n_cdofs &&
        a->n_sblk == b->n_sblk && a->fd == b->fd && a->cdofs == b->cdofs))
    return false;
  return is_f64(a) ? same_inst_shape<double>(a, b) : same_inst_shape<float>(a, b);
}

extern "C" int nmr_pool_attach(nmr_pool* p, nmr_inst* in, int* slot) {
  if (!p || !in || !slot || in->ctx != p->ctx) return fail(NMR_ERR_ARG, "bad argument");
  if (in->pool) return fail(NMR_ERR_ARG, "instance is already attached to a pool");
  CHK(set_device(p->ctx));
  if (p->proto && !same_class(p->proto, in)) return fail(NMR_ERR_ARG, "instance does not match the pool's class");
  int s = -1;
  for (int k = 0; k < p->capacity; ++k)
    if (!p->slots[k]) {
      s = k;
      break;
    }
  if (s < 0) return fail(NMR_ERR_BUDGET, "pool is full");
  if (!p->proto) {
    p->proto_copy = *in;
    p->proto_copy.step_graphs.clear();
    p->proto_copy.pool = nullptr;
    p->proto = &p->proto_copy;
    p->proto->dec->refs++;  // the pool's graph references the decoder's weights
    p->isz = is_f64(in) ? sizeof(Inst<double>) : sizeof(Inst<float>);
    std::vector<unsigned char> zero(p->isz * p->capacity, 0);  // active = 0 everywhere
    HIPCHK(hipMalloc(&p->tab, zero.size()));
    HIPCHK(hipMemcpy(p->tab, zero.data(), zero.size(), hipMemcpyHostToDevice));
    if (in->gram && in->n_cdofs > 0) {
      HIPCHK(hipMalloc(&p->rows, in->cdofs.size() * sizeof(int)));
      HIPCHK(hipMemcpy(p->rows, in->cdofs.data(), in->cdofs.size() * sizeof(int), hipMemcpyHostToDevice));
    }
  }
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  HIPCHK(hipMemcpy(static_cast<unsigned char*>(p->tab) + s * p->isz, in->host.data(), p->isz,
                   hipMemcpyHostToDevice));
  p->slots[s] = in;
  in->pool = p;
  in->pool_slot = s;
  *slot = s;
  return NMR_OK;
}

extern "C" int nmr_pool_detach(nmr_pool* p, int s) {
  if (!p || s < 0 || s >= p->capacity || !p->slots[s]) return fail(NMR_ERR_ARG, "bad slot");
  CHK(set_device(p->ctx));
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  const int zero = 0;  // Inst<T>::active is the first member
  HIPCHK(hipMemcpy(static_cast<unsigned char*>(p->tab) + s * p->isz, &zero, sizeof(int), hipMemcpyHostToDevice));
  p->slots[s]->pool = nullptr;
  p->slots[s]->pool_slot = -1;
  p->slots[s] = nullptr;
  return NMR_OK;
}

extern "C" int nmr_pool_step(nmr_pool* p, int n_iters, int* status, float* ms) {
  if (!p) return fail(NMR_ERR_ARG, "null pool");
  if (n_iters < 1 || n_iters > kMaxIters) return fail(NMR_ERR_ARG, "n_iters must be in [1, 64]");
  if (!p->proto) return NMR_OK;  // nothing ever attached
  nmr_ctx* c = p->ctx;
  CHK(set_device(c));
  if (p->tile_epoch != c->tile_epoch) {
    pool_drop_graphs(p);
    p->tile_epoch = c->tile_epoch;
  }
  auto it = p->graphs.find(n_iters);
  if (it == p->graphs.end()) {
    Group g = group_of({p->proto}, p->tab);
    g.nb = p->capacity;
    // every member shares the class's rows (nmr_pool_attach checks them), but a
    // table entry of an empty slot may be stale: only kernels that take the
    // rows from the pool's own copy and never follow an empty slot's pointers
    // use them (the paired output layer, the batched output-layer
    // backpropagation)
    g.same_rows = false;
    g.rows = p->proto->gram ? p->rows : nullptr;
    g.n_rows = p->proto->n_cdofs;
    int live = 0;
    for (nmr_inst* x : p->slots) live += x != nullptr;
    CHK(choose_tiles(c, g, 2 * live >= p->capacity));
    hipGraphExec_t ex;
    CHK(capture(c, {g}, n_iters, &ex));
    it = p->graphs.emplace(n_iters, ex).first;
  }
  if (ms) HIPCHK(hipEventRecord(c->ev[0], c->stream));
  HIPCHK(hipGraphLaunch(it->second, c->stream));
  if (ms) {
    HIPCHK(hipEventRecord(c->ev[1], c->stream));
    HIPCHK(hipEventSynchronize(c->ev[1]));
    HIPCHK(hipEventElapsedTime(ms, c->ev[0], c->ev[1]));
  }
  if (status) {
    for (int k = 0; k < p->capacity; ++k) {
      status[k] = 0;
      if (p->slots[k]) {
        int st;
        CHK(read_status(p->slots[k], &st));
        status[k] = map_status(st);
      }
    }
  }
  return NMR_OK;
}

extern "C" int nmr_instance_status(nmr_inst* in) {
  if (!in) return fail(NMR_ERR_ARG, "null instance");
  CHK(set_device(in->ctx));
  int st;
  CHK(read_status(in, &st));
  return map_status(st);
}

// ---------------------------------------------------------------------------
// measurement: replay one phase between events (state saved and restored)
// ---------------------------------------------------------------------------
template <typename T>
static void enqueue_phase(const Group& g, int phase, hipStream_t s) {
  const Inst<T>* tab = static_cast<const Inst<T>*>(g.tab);
  const DecoderDev& d = g.dec->d;
  switch (phase) {
    case NMR_PHASE_DEC_HIDDEN:
      for (int l = 0; l < d.L - 1; ++l) launch_fwd_hidden<T>(d, l, tab, g.nb, g.Cp, g.fd, g.tf[l], s);
      break;
    case NMR_PHASE_DEC_OUT:
      launch_fwd_out<T>(d, tab, g.nb, g.gram ? g.max_cdofs : g.maxN, out_channels(g), g.same_rows,
                        g.gram ? g.rows : nullptr, s);
      if (g.any_np) launch_filter<T>(tab, g.nb, g.maxN, 1, s);
      break;
    case NMR_PHASE_CUBATURE: launch_cubature<T>(tab, g.nb, g.max_cblk, g.maxR, s); break;
    case NMR_PHASE_MASS:
      if (g.gram) launch_gram<T>(tab, g.nb, g.n_gblk, g.K, g.n_q, s);
      else launch_mass<T>(tab, g.nb, g.max_mblk, g.maxR, g.n_q, s);
      break;
    case NMR_PHASE_SUMS: launch_sums<T>(tab, g.nb, g.max_entries, g.max_cblk, s); break;
    case NMR_PHASE_BWD_OUT: launch_bwd_out<T>(d, tab, g.nb, g.gram ? g.max_sblk : g.max_bblk, s); break;
    case NMR_PHASE_BWD_HIDDEN:
      launch_bwd_reduce<T>(d, tab, g.nb, s);
      for (int l = d.L - 2; l >= 0; --l) launch_bwd_hidden<T>(d, l, tab, g.nb, g.Cb, g.fd, g.tb[l], s);
      break;
    case NMR_PHASE_SOLVE: launch_solve<T>(tab, g.nb, 0, SOLVE_UPDATE, nullptr, nullptr, s); break;
    default: break;
  }
}

template <typename T>
static int time_phase_impl(nmr_inst* in, int phase, int reps, float* avg_us) {
  nmr_ctx* c = in->ctx;
  Inst<T>& I = host_inst<T>(in);
  const int R = in->R, nq = in->n_q;
  std::vector<double> save(3 * R + 3 * nq);
  int st = 0;
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(save.data(), I.r, R * 8, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(save.data() + R, I.rbar, R * 8, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(save.data() + 2 * R, I.rdot, R * 8, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(save.data() + 3 * R, I.dec_in, 3 * nq * 8, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&st, I.status, sizeof(int), hipMemcpyDeviceToHost));
  std::vector<nmr_inst*> v{in};
  Group g = group_of(v, in->tab);
  enqueue_phase<T>(g, phase, c->stream);
  HIPCHK(hipEventRecord(c->ev[0], c->stream));
  for (int k = 0; k < reps; ++k) enqueue_phase<T>(g, phase, c->stream);
  HIPCHK(hipEventRecord(c->ev[1], c->stream));
  HIPCHK(hipEventSynchronize(c->ev[1]));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
  *avg_us = 1000.f * ms / reps;
  HIPCHK(hipMemcpy(I.r, save.data(), R * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(I.rbar, save.data() + R, R * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(I.rdot, save.data() + 2 * R, R * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(I.dec_in, save.data() + 3 * R, 3 * nq * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(I.status, &st, sizeof(int), hipMemcpyHostToDevice));
  return NMR_OK;
}

extern "C" int nmr_time_phase(nmr_inst* in, int phase, int reps, float* avg_us) {
  if (!in || !avg_us || phase < 0 || phase >= NMR_PHASE_COUNT || reps < 1) return fail(NMR_ERR_ARG, "bad argument");
  CHK(set_device(in->ctx));
  return is_f64(in) ? time_phase_impl<double>(in, phase, reps, avg_us) : time_phase_impl<float>(in, phase, reps, avg_us);
}

// ---------------------------------------------------------------------------
// neural cubature training (Sec. 5): training data from the instance's
// decoder and mesh, then the alternation of the weight and selection nets
// ---------------------------------------------------------------------------
namespace {

// every tet of the instance's mesh in FP64, rest shape on the device
int mesh_build(nmr_inst* in, DevMem& M, TrainMesh* tm) {
  tm->n = in->n;
  tm->N = in->N;
  tm->m = in->m;
  if (is_f64(in)) {
    tm->mu = host_inst<double>(in).mu;
    tm->lam = host_inst<double>(in).lam;
  } else {
    tm->mu = host_inst<float>(in).mu;
    tm->lam = host_inst<float>(in).lam;
  }
  double *X, *Bm, *Ve;
  int* tets;
  CHK(dalloc_t(M, 3 * (size_t)in->n, &X));
  CHK(dalloc_t(M, 4 * (size_t)in->m, &tets));
  CHK(dalloc_t(M, 9 * (size_t)in->m, &Bm));
  CHK(dalloc_t(M, (size_t)in->m, &Ve));
  HIPCHK(hipMemcpy(X, in->Xh.data(), 3 * (size_t)in->n * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(tets, in->tets_h.data(), 4 * (size_t)in->m * sizeof(int), hipMemcpyHostToDevice));
  launch_rest_all(X, tets, in->m, Bm, Ve, in->ctx->stream);
  HIPCHK(hipGetLastError());
  tm->X = X;
  tm->tets = tets;
  tm->Bm = Bm;
  tm->Ve = Ve;
  return NMR_OK;
}

// F[p] (m x R), u[p] (N) for poses r[p] (device, P x R), p < P; then f[p] = sum_e F[p][e]
template <typename T>
int pose_forces(nmr_inst* in, const TrainMesh& tm, const double* r, int P, double* u, double* F, double* f) {
  nmr_ctx* c = in->ctx;
  hipStream_t s = c->stream;
  Inst<T>& I = host_inst<T>(in);
  const int N = in->N, nq = in->n_q, np = in->n_p, R = in->R;
  DevMem tmp;
  T *uD, *J, *dJ, *Hdd;
  int* st;
  std::vector<double> save(3 * nq);
  int rc = NMR_OK;
  auto body = [&]() -> int {
    CHK(dalloc_t(tmp, N, &uD));
    CHK(dalloc_t(tmp, (size_t)N * nq, &J));
    CHK(dalloc_t(tmp, (size_t)N * nq, &dJ));
    CHK(dalloc_t(tmp, N, &Hdd));
    CHK(dalloc_t(tmp, 1, &st));
    // the decoder input buffer is the instance's: kept and put back
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(save.data(), I.dec_in, 3 * nq * sizeof(double), hipMemcpyDeviceToHost));
    void* dt_tab;
    CHK(direct_tab<T>(in, &dt_tab));
    const Inst<T>* tab = static_cast<const Inst<T>*>(dt_tab);
    std::vector<nmr_inst*> v{in};
    Group g = group_of(v, dt_tab);
    g.gram = false;
    for (int p = 0; p < P; ++p) {
      const double* rp = r + (size_t)p * R;
      HIPCHK(hipMemcpyAsync(I.dec_in, rp + np, nq * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemsetAsync(I.dec_in + nq, 0, 2 * nq * sizeof(double), s));
      enqueue_decoder_fwd<T>(g, s, 0);
      launch_unpack<T>(tab, uD, J, dJ, Hdd, N, s);
      launch_elem_forces<T>(tm, I.U, np, rp, uD, J, nq, u + (size_t)p * N, F + (size_t)p * tm.m * R, st, s);
    }
    if (f) launch_force_sum(F, P, tm.m, R, f, s);
    HIPCHK(hipGetLastError());
    int hst = 0;
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(&hst, st, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(I.dec_in, save.data(), 3 * nq * sizeof(double), hipMemcpyHostToDevice));
    if (hst & ST_INVERTED) return fail(NMR_ERR_INVERTED, "a tet has det F <= 0 at a training pose");
    return NMR_OK;
  };
  rc = body();
  (void)hipStreamSynchronize(s);
  tmp.release();
  return rc;
}

}  // namespace

extern "C" int nmr_element_forces(nmr_inst* in, const double* r, double* F, double* f_or_null, double* u_or_null) {
  if (!in || !r || !F) return fail(NMR_ERR_ARG, "null argument");
  CHK(set_device(in->ctx));
  DevMem M;
  TrainMesh tm{};
  double* u = u_or_null;
  int rc = mesh_build(in, M, &tm);
  if (rc == NMR_OK && !u) rc = dalloc_t(M, (size_t)in->N, &u);
  if (rc == NMR_OK)
    rc = is_f64(in) ? pose_forces<double>(in, tm, r, 1, u, F, f_or_null)
                    : pose_forces<float>(in, tm, r, 1, u, F, f_or_null);
  (void)hipStreamSynchronize(in->ctx->stream);
  M.release();
  return rc;
}

struct nmr_trainer {
  nmr_ctx* ctx = nullptr;
  DevMem dev;
  int P = 0, R = 0, n = 0, N = 0, m = 0;
  int K = 0, epochs = 0, c_max = 0, nC = 0;
  double lr = 1e-3, b1 = 0.9, b2 = 0.999, eps = 1e-8;
  long long tw = 0, ts = 0;  // Adam steps taken by each net
  size_t n_w = 0;            // weight-net parameter count
  TrainMesh tm{};
  TrainData td{};
  WNetDev w{};
  SNetDev sd{};
  double *wm = nullptr, *wv = nullptr, *sm = nullptr, *sv = nullptr;
  double* theta = nullptr;
  double* mean = nullptr;    // [m] averaged scores (also the sampling distances)
  int* C = nullptr;
  int* inC = nullptr;
  double* losses = nullptr;  // [2 epochs] one alternation's loss history
  std::vector<int> Ch;       // host copy of C
  int broken = 0;            // 1 after a selection found no finite score
};

namespace {

int trainer_build(nmr_inst* in, const nmr_cubature_train_desc* d, nmr_trainer* tr) {
  DevMem& M = tr->dev;
  const int P = d->n_poses, R = in->R, n = in->n, N = in->N, m = in->m;
  tr->P = P;
  tr->R = R;
  tr->n = n;
  tr->N = N;
  tr->m = m;
  tr->K = d->K;
  tr->epochs = d->epochs;
  tr->c_max = d->c_max;
  tr->lr = d->lr;
  tr->b1 = d->beta1;
  tr->b2 = d->beta2;
  tr->eps = d->eps;
  CHK(mesh_build(in, M, &tr->tm));
  // training data
  double *r, *F, *f, *fb, *u, *loss_p;
  CHK(dalloc_t(M, (size_t)P * R, &r));
  CHK(dalloc_t(M, (size_t)P * m * R, &F));
  CHK(dalloc_t(M, (size_t)P * R, &f));
  CHK(dalloc_t(M, (size_t)P * R, &fb));
  CHK(dalloc_t(M, (size_t)P * N, &u));
  CHK(dalloc_t(M, (size_t)P, &loss_p));
  CHK(dalloc_t(M, (size_t)d->c_max, &tr->C));
  CHK(dalloc_t(M, (size_t)m, &tr->inC));
  CHK(dalloc_t(M, (size_t)m, &tr->mean));
  CHK(dalloc_t(M, 2 * (size_t)d->epochs, &tr->losses));
  HIPCHK(hipMemcpy(r, d->poses, (size_t)P * R * sizeof(double), hipMemcpyHostToDevice));
  CHK(is_f64(in) ? pose_forces<double>(in, tr->tm, r, P, u, F, f) : pose_forces<float>(in, tr->tm, r, P, u, F, f));
  tr->td = TrainData{P, R, m, r, F, f, fb, tr->C, loss_p};
  // weight net
  const nmr_mlp_desc* wd = d->wnet;
  WNetDev& w = tr->w;
  w.L = wd->n_layers;
  w.scale = d->wnet_scale;
  size_t off = 0;
  for (int l = 0; l <= w.L; ++l) w.width[l] = wd->widths[l];
  for (int l = 0; l < w.L; ++l) {
    w.Woff[l] = off;
    off += (size_t)w.width[l + 1] * w.width[l];
    w.boff[l] = off;
    off += (size_t)w.width[l + 1];
  }
  tr->n_w = off;
  CHK(dalloc_t(M, off, &w.x));
  CHK(dalloc_t(M, off, &w.g));
  CHK(dalloc_t(M, off, &tr->wm));
  CHK(dalloc_t(M, off, &tr->wv));
  {
    std::vector<double> hx(off);
    for (int l = 0; l < w.L; ++l) {
      std::copy(wd->W[l], wd->W[l] + (size_t)w.width[l + 1] * w.width[l], hx.begin() + w.Woff[l]);
      std::copy(wd->b[l], wd->b[l] + w.width[l + 1], hx.begin() + w.boff[l]);
    }
    HIPCHK(hipMemcpy(w.x, hx.data(), off * sizeof(double), hipMemcpyHostToDevice));
  }
  for (int l = 0; l < w.L; ++l) {
    CHK(dalloc_t(M, (size_t)P * w.width[l + 1], &w.a[l]));
    CHK(dalloc_t(M, (size_t)P * w.width[l + 1], &w.z[l]));
    CHK(dalloc_t(M, (size_t)P * w.width[l + 1], &w.d[l]));
  }
  // selection net: one-ring graph (self included) and vertex -> tet lists
  std::vector<std::vector<int>> ring(n);
  for (int e = 0; e < m; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) ring[in->tets_h[4 * e + a]].push_back(in->tets_h[4 * e + b]);
  std::vector<int> gptr(n + 1, 0), gidx;
  std::vector<double> gval;
  for (int i = 0; i < n; ++i) {
    std::sort(ring[i].begin(), ring[i].end());
    ring[i].erase(std::unique(ring[i].begin(), ring[i].end()), ring[i].end());
    gptr[i + 1] = gptr[i] + (int)ring[i].size();
  }
  for (int i = 0; i < n; ++i)
    for (int j : ring[i]) {
      gidx.push_back(j);
      gval.push_back(1.0 / std::sqrt((double)ring[i].size() * (double)ring[j].size()));
    }
  std::vector<int> vptr(n + 1, 0), vtet(4 * (size_t)m);
  for (int e = 0; e < m; ++e)
    for (int a = 0; a < 4; ++a) vptr[in->tets_h[4 * e + a] + 1]++;
  for (int i = 0; i < n; ++i) vptr[i + 1] += vptr[i];
  {
    std::vector<int> fill(vptr.begin(), vptr.end() - 1);
    for (int e = 0; e < m; ++e)
      for (int a = 0; a < 4; ++a) vtet[fill[in->tets_h[4 * e + a]]++] = e;
  }
  SNetDev& sd = tr->sd;
  sd.n = n;
  sd.m = m;
  sd.R = R;
  sd.P = P;
  sd.nbv = (n + 255) / 256;
  sd.nbe = (m + NMR_TRAIN_SBE - 1) / NMR_TRAIN_SBE;
  sd.u = u;
  int *g_ptr, *g_idx, *vt_ptr, *vt_tet;
  double* g_val;
  CHK(dalloc_t(M, (size_t)n + 1, &g_ptr));
  CHK(dalloc_t(M, gidx.size(), &g_idx));
  CHK(dalloc_t(M, gval.size(), &g_val));
  CHK(dalloc_t(M, (size_t)n + 1, &vt_ptr));
  CHK(dalloc_t(M, vtet.size(), &vt_tet));
  HIPCHK(hipMemcpy(g_ptr, gptr.data(), gptr.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(g_idx, gidx.data(), gidx.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(g_val, gval.data(), gval.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(vt_ptr, vptr.data(), vptr.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(vt_tet, vtet.data(), vtet.size() * sizeof(int), hipMemcpyHostToDevice));
  sd.g_ptr = g_ptr;
  sd.g_idx = g_idx;
  sd.g_val = g_val;
  sd.vt_ptr = vt_ptr;
  sd.vt_tet = vt_tet;
  sd.tets = tr->tm.tets;
  sd.inC = tr->inC;
  CHK(dalloc_t(M, 170, &tr->theta));
  CHK(dalloc_t(M, 170, &tr->sm));
  CHK(dalloc_t(M, 170, &tr->sv));
  HIPCHK(hipMemcpy(tr->theta, d->snet, 170 * sizeof(double), hipMemcpyHostToDevice));
  sd.theta = tr->theta;
  sd.F = F;
  sd.fb = fb;
  // poses per chunk: every pose at once up to 4 GiB of per-pose intermediates
  const size_t per_pose = (51 * (size_t)n + 8 * (size_t)m) * sizeof(double);
  sd.nc = d->pose_chunk > 0 ? std::min(d->pose_chunk, P)
                            : (int)std::max<size_t>(1, std::min<size_t>(P, (size_t(4) << 30) / per_pose));
  sd.p0 = 0;
  const int nc = sd.nc;
  const size_t Pn = (size_t)nc * n;
  CHK(dalloc_t(M, 3 * Pn, &sd.H0));
  CHK(dalloc_t(M, 8 * Pn, &sd.P1));
  CHK(dalloc_t(M, 8 * Pn, &sd.X1));
  CHK(dalloc_t(M, 8 * Pn, &sd.H1));
  CHK(dalloc_t(M, 8 * Pn, &sd.P2));
  CHK(dalloc_t(M, 8 * Pn, &sd.X2));
  CHK(dalloc_t(M, 8 * Pn, &sd.T2));
  CHK(dalloc_t(M, (size_t)P * m, &sd.z));
  CHK(dalloc_t(M, (size_t)nc * sd.nbe * (R + 2), &sd.pf));
  CHK(dalloc_t(M, (size_t)P * 8, &sd.pstat));
  CHK(dalloc_t(M, (size_t)P * R, &sd.res));
  sd.loss_p = loss_p;
  CHK(dalloc_t(M, (size_t)nc * m * 8, &sd.dg));
  CHK(dalloc_t(M, (size_t)nc * sd.nbe * 81, &sd.pe));
  CHK(dalloc_t(M, (size_t)nc * sd.nbv * 64, &sd.pv2));
  CHK(dalloc_t(M, (size_t)nc * sd.nbv * 24, &sd.pv1));
  CHK(dalloc_t(M, (size_t)P * 170, &sd.gpose));
  CHK(dalloc_t(M, 170, &sd.grad));
  // initial cubature set: the caller's, or farthest-point samples
  if (d->c0) {
    std::vector<int> hin(m, 0);
    for (int k = 0; k < d->n_c0; ++k) {
      const int e = d->c0[k];
      if (e < 0 || e >= m) return fail(NMR_ERR_ARG, "initial cubature id out of range");
      if (hin[e]) return fail(NMR_ERR_ARG, "initial cubature ids must be distinct");
      hin[e] = 1;
    }
    HIPCHK(hipMemcpy(tr->C, d->c0, d->n_c0 * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(tr->inC, hin.data(), m * sizeof(int), hipMemcpyHostToDevice));
  } else {
    launch_fps(tr->tm.X, tr->tm.tets, m, d->n_c0, tr->mean, tr->C, tr->inC, in->ctx->stream);
    HIPCHK(hipGetLastError());
  }
  tr->nC = d->n_c0;
  tr->Ch.resize(d->c_max);
  HIPCHK(hipStreamSynchronize(in->ctx->stream));
  HIPCHK(hipMemcpy(tr->Ch.data(), tr->C, d->n_c0 * sizeof(int), hipMemcpyDeviceToHost));
  for (int k = 0; k < d->n_c0; ++k)
    if (tr->Ch[k] < 0) return fail(NMR_ERR_NONFINITE, "non-finite tet centroids");
  return NMR_OK;
}

int trainer_alternation(nmr_trainer* tr, double* lw, double* ls, int* added) {
  hipStream_t s = tr->ctx->stream;
  const int E = tr->epochs;
  for (int ep = 0; ep < E; ++ep) {
    WNetDev w = tr->w;
    w.loss_out = tr->losses + ep;
    launch_wnet_epoch(w, tr->td, tr->nC, 0, s);
    ++tr->tw;
    launch_adam(tr->w.x, tr->w.g, tr->wm, tr->wv, (long long)tr->n_w, tr->lr, tr->b1, tr->b2, tr->eps,
                1.0 - std::pow(tr->b1, (double)tr->tw), 1.0 - std::pow(tr->b2, (double)tr->tw), s);
  }
  launch_wnet_epoch(tr->w, tr->td, tr->nC, 1, s);  // residual forces fb with the trained weights
  for (int ep = 0; ep < E; ++ep) {
    SNetDev sd = tr->sd;
    sd.loss_out = tr->losses + E + ep;
    launch_snet_epoch(sd, s);
    ++tr->ts;
    launch_adam(tr->theta, tr->sd.grad, tr->sm, tr->sv, 170, tr->lr, tr->b1, tr->b2, tr->eps,
                1.0 - std::pow(tr->b1, (double)tr->ts), 1.0 - std::pow(tr->b2, (double)tr->ts), s);
  }
  launch_snet_forward(tr->sd, s);  // scores with the trained selection net
  launch_select(tr->sd, tr->mean, tr->K, tr->inC, tr->C, tr->nC, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  if (lw) HIPCHK(hipMemcpy(lw, tr->losses, E * sizeof(double), hipMemcpyDeviceToHost));
  if (ls) HIPCHK(hipMemcpy(ls, tr->losses + E, E * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(tr->Ch.data() + tr->nC, tr->C + tr->nC, tr->K * sizeof(int), hipMemcpyDeviceToHost));
  if (added) std::copy(tr->Ch.begin() + tr->nC, tr->Ch.begin() + tr->nC + tr->K, added);
  for (int k = 0; k < tr->K; ++k)
    if (tr->Ch[tr->nC + k] < 0) {
      tr->broken = 1;
      return fail(NMR_ERR_NONFINITE, "no finite candidate score: the trainer is left unusable");
    }
  tr->nC += tr->K;
  return NMR_OK;
}

}  // namespace

extern "C" int nmr_trainer_create(nmr_inst* in, const nmr_cubature_train_desc* d, nmr_trainer** out) {
  if (!in || !d || !out) return fail(NMR_ERR_ARG, "null argument");
  *out = nullptr;
  if (d->n_poses < 1 || !d->poses) return fail(NMR_ERR_ARG, "need at least one pose");
  if (d->K < 1 || d->epochs < 1) return fail(NMR_ERR_ARG, "K and epochs must be >= 1");
  if (!(d->lr > 0.0) || !(d->beta1 >= 0.0 && d->beta1 < 1.0) || !(d->beta2 >= 0.0 && d->beta2 < 1.0) ||
      !(d->eps > 0.0))
    return fail(NMR_ERR_ARG, "Adam needs lr > 0, 0 <= beta < 1, eps > 0");
  if (!d->snet) return fail(NMR_ERR_ARG, "missing selection-net parameters");
  CHK(check_mlp(d->wnet, 1, "weight net"));
  const nmr_mlp_desc* wd = d->wnet;
  if (wd->widths[0] != in->R) return fail(NMR_ERR_ARG, "weight net input must be R");
  if (wd->widths[wd->n_layers] != d->c_max) return fail(NMR_ERR_ARG, "weight net output must be c_max");
  for (int l = 1; l < wd->n_layers; ++l)
    if (wd->widths[l] > 1024) return fail(NMR_ERR_ARG, "weight-net hidden widths must be <= 1024");
  if (d->n_c0 < 1 || d->n_c0 > d->c_max) return fail(NMR_ERR_ARG, "need 1 <= n_c0 <= c_max");
  if (d->c_max >= in->m) return fail(NMR_ERR_ARG, "c_max must be below the tet count");
  if (!(d->wnet_scale > 0.0)) return fail(NMR_ERR_ARG, "wnet_scale must be > 0");
  if (d->pose_chunk < 0) return fail(NMR_ERR_ARG, "pose_chunk must be >= 0");
  CHK(set_device(in->ctx));
  nmr_trainer* tr = new nmr_trainer();
  tr->ctx = in->ctx;
  int rc = trainer_build(in, d, tr);
  nmr_ctx* c = in->ctx;
  if (rc == NMR_OK && c->budget && c->used + tr->dev.bytes > c->budget) rc = fail(NMR_ERR_BUDGET, "trainer exceeds HBM budget");
  if (rc != NMR_OK) {
    (void)hipStreamSynchronize(c->stream);
    tr->dev.release();
    delete tr;
    return rc;
  }
  c->used += tr->dev.bytes;
  *out = tr;
  return NMR_OK;
}

extern "C" int nmr_trainer_destroy(nmr_trainer* tr) {
  if (!tr) return fail(NMR_ERR_ARG, "null trainer");
  CHK(set_device(tr->ctx));
  (void)hipStreamSynchronize(tr->ctx->stream);
  tr->ctx->used -= tr->dev.bytes;
  tr->dev.release();
  delete tr;
  return NMR_OK;
}

extern "C" int nmr_trainer_run(nmr_trainer* tr, int n_alternations, double* loss_w, double* loss_s, int* added,
                               float* ms_or_null) {
  if (!tr || n_alternations < 0) return fail(NMR_ERR_ARG, "bad argument");
  if (tr->broken) return fail(NMR_ERR_NONFINITE, "an earlier selection failed");
  if (tr->nC + (long long)n_alternations * tr->K > tr->c_max)
    return fail(NMR_ERR_ARG, "the cubature set would exceed c_max");
  CHK(set_device(tr->ctx));
  nmr_ctx* c = tr->ctx;
  HIPCHK(hipEventRecord(c->ev[0], c->stream));
  for (int a = 0; a < n_alternations; ++a)
    CHK(trainer_alternation(tr, loss_w ? loss_w + (size_t)a * tr->epochs : nullptr,
                            loss_s ? loss_s + (size_t)a * tr->epochs : nullptr,
                            added ? added + (size_t)a * tr->K : nullptr));
  HIPCHK(hipEventRecord(c->ev[1], c->stream));
  HIPCHK(hipEventSynchronize(c->ev[1]));
  if (ms_or_null) HIPCHK(hipEventElapsedTime(ms_or_null, c->ev[0], c->ev[1]));
  return NMR_OK;
}

extern "C" int nmr_trainer_get(nmr_trainer* tr, int* n_c, int32_t* C_or_null, double* wnet_or_null,
                               double* snet_or_null) {
  if (!tr || !n_c) return fail(NMR_ERR_ARG, "null argument");
  CHK(set_device(tr->ctx));
  HIPCHK(hipStreamSynchronize(tr->ctx->stream));
  *n_c = tr->nC;
  if (C_or_null) std::copy(tr->Ch.begin(), tr->Ch.begin() + tr->nC, C_or_null);
  if (wnet_or_null) HIPCHK(hipMemcpy(wnet_or_null, tr->w.x, tr->n_w * sizeof(double), hipMemcpyDeviceToHost));
  if (snet_or_null) HIPCHK(hipMemcpy(snet_or_null, tr->theta, 170 * sizeof(double), hipMemcpyDeviceToHost));
  return NMR_OK;
}

extern "C" int nmr_trainer_pose(nmr_trainer* tr, int p, double* F_or_null, double* f_or_null, double* u_or_null) {
  if (!tr || p < 0 || p >= tr->P) return fail(NMR_ERR_ARG, "bad argument");
  CHK(set_device(tr->ctx));
  HIPCHK(hipStreamSynchronize(tr->ctx->stream));
  const size_t mR = (size_t)tr->m * tr->R;
  if (F_or_null) HIPCHK(hipMemcpy(F_or_null, tr->td.F + p * mR, mR * sizeof(double), hipMemcpyDeviceToHost));
  if (f_or_null)
    HIPCHK(hipMemcpy(f_or_null, tr->td.f + (size_t)p * tr->R, tr->R * sizeof(double), hipMemcpyDeviceToHost));
  if (u_or_null)
    HIPCHK(hipMemcpy(u_or_null, tr->sd.u + (size_t)p * tr->N, tr->N * sizeof(double), hipMemcpyDeviceToHost));
  return NMR_OK;
}

extern "C" int nmr_trainer_time_phase(nmr_trainer* tr, int phase, int reps, float* avg_us) {
  if (!tr || !avg_us || reps < 1 || phase < 0 || phase >= NMR_TRAIN_PHASE_COUNT) return fail(NMR_ERR_ARG, "bad argument");
  if (tr->broken) return fail(NMR_ERR_NONFINITE, "an earlier selection failed");
  CHK(set_device(tr->ctx));
  nmr_ctx* c = tr->ctx;
  hipStream_t s = c->stream;
  // valid inputs for every phase: residual forces of the current weights and
  // a selection-net forward pass (intermediates only; no parameter changes)
  launch_wnet_epoch(tr->w, tr->td, tr->nC, 1, s);
  launch_snet_forward(tr->sd, s);
  auto once = [&]() {
    WNetDev w = tr->w;
    SNetDev sd = tr->sd;
    w.loss_out = tr->losses;
    sd.loss_out = tr->losses + tr->epochs;
    switch (phase) {
      case NMR_TRAIN_PHASE_S_EPOCH: launch_snet_epoch(sd, s); break;
      case NMR_TRAIN_PHASE_W_EPOCH: launch_wnet_epoch(w, tr->td, tr->nC, 0, s); break;
      case NMR_TRAIN_PHASE_S_ELEM_FWD: launch_snet_elem(sd, 0, s); break;
      default: launch_snet_elem(sd, 1, s); break;
    }
  };
  once();
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(c->ev[0], s));
  for (int k = 0; k < reps; ++k) once();
  HIPCHK(hipEventRecord(c->ev[1], s));
  HIPCHK(hipEventSynchronize(c->ev[1]));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
  *avg_us = 1000.f * ms / reps;
  return NMR_OK;
}
