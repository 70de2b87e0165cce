// C ABI of the library: layouts, device problems, ORAS application and the
// FGMRES driver (Sec. 4-5 of the paper).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "kernels.h"
#include "mxw_internal.h"

namespace mxw {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

// ---------------------------------------------------------------------------
// kernel timing with HIP events on the launching stream
// ---------------------------------------------------------------------------
struct TimingRec {
  std::string name;
  hipEvent_t a, b;
};
static std::mutex g_tmu;
static bool g_timing = false;
static thread_local bool g_capturing = false;   // no timers inside a captured graph
static std::vector<TimingRec> g_pending;
static std::vector<hipEvent_t> g_event_pool;   // events reused across launches
static std::map<std::string, std::pair<double, int64_t>> g_totals;

static hipEvent_t pooled_event() {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Range timer: events recorded on the stream around a group of launches.
struct ScopedTimer {
  hipStream_t st;
  const char* name;
  hipEvent_t a = nullptr, b = nullptr;
  ScopedTimer(hipStream_t s, const char* n) : st(s), name(n) {
    if (!g_timing || g_capturing) return;
    a = pooled_event();
    b = pooled_event();
    if (!a || !b) {
      a = b = nullptr;
      return;
    }
    hipEventRecord(a, st);
  }
  ~ScopedTimer() {
    if (!a) return;
    hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_tmu);
    g_pending.push_back({name, a, b});
  }
};

// Kernel timer: the next launch in scope carries the start/stop events in its
// own dispatch (hipExtLaunchKernelGGL), so timing adds no packets to the stream.
struct KernelEvents {
  hipEvent_t a = nullptr, b = nullptr;
  bool used = false;
};
static thread_local KernelEvents* g_kernel_events = nullptr;

bool take_timer_events(hipEvent_t* a, hipEvent_t* b) {
  KernelEvents* k = g_kernel_events;
  if (!k || k->used || !k->a) return false;
  k->used = true;
  *a = k->a;
  *b = k->b;
  return true;
}

struct ScopedKernelTimer {
  const char* name;
  KernelEvents ev;
  explicit ScopedKernelTimer(const char* n) : name(n) {
    if (!g_timing || g_capturing) return;
    ev.a = pooled_event();
    ev.b = pooled_event();
    if (!ev.a || !ev.b) {
      ev.a = ev.b = nullptr;
      return;
    }
    g_kernel_events = &ev;
  }
  ~ScopedKernelTimer() {
    if (!ev.a) return;
    g_kernel_events = nullptr;
    std::lock_guard<std::mutex> lk(g_tmu);
    if (ev.used) {
      g_pending.push_back({name, ev.a, ev.b});
    } else {
      g_event_pool.push_back(ev.a);
      g_event_pool.push_back(ev.b);
    }
  }
};

static void flush_timing();

// Recorded timing events keep the launches they were recorded with alive in
// the runtime, and with them the device buffers those launches used: a freed
// buffer is only returned once they go.  Before a problem releases its memory
// the pending records are folded into the totals and the pooled events
// destroyed (new ones are created on demand).
static void release_timing_events() {
  flush_timing();
  std::lock_guard<std::mutex> lk(g_tmu);
  for (hipEvent_t e : g_event_pool) hipEventDestroy(e);
  g_event_pool.clear();
}

static void flush_timing() {
  std::lock_guard<std::mutex> lk(g_tmu);
  for (auto& r : g_pending) {
    hipEventSynchronize(r.b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, r.a, r.b);
    auto& t = g_totals[r.name];
    t.first += ms;
    t.second += 1;
    g_event_pool.push_back(r.a);
    g_event_pool.push_back(r.b);
  }
  g_pending.clear();
}

// ---------------------------------------------------------------------------
// device memory: every allocation goes through a context (the caller's
// allocator callback and HBM budget, or hipMalloc with no budget), which
// counts the bytes in use and their peak
// ---------------------------------------------------------------------------
struct CtxState {
  int device = 0;
  uint64_t budget = 0;   // 0: no limit
  mxw_alloc_fn alloc = nullptr;
  mxw_free_fn free_ = nullptr;
  void* user = nullptr;
  std::mutex mu;
  uint64_t in_use = 0, peak = 0;
  int64_t live = 0;      // allocations not yet returned

  bool reserve(uint64_t bytes, std::string* why) {
    std::lock_guard<std::mutex> lk(mu);
    if (budget && in_use + bytes > budget) {
      std::ostringstream os;
      os << "HBM budget exceeded: " << in_use << " bytes in use + " << bytes << " requested > budget " << budget;
      *why = os.str();
      return false;
    }
    in_use += bytes;
    peak = std::max(peak, in_use);
    ++live;
    return true;
  }
  void unreserve(uint64_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    in_use -= bytes;
    --live;
  }
};

// the context of calls made without one: hipMalloc / hipFree, no budget,
// the current device
static std::shared_ptr<CtxState> default_ctx() {
  static std::shared_ptr<CtxState> d = [] {
    auto c = std::make_shared<CtxState>();
    c->device = -1;
    return c;
  }();
  return d;
}

struct DevMem {
  std::shared_ptr<CtxState> ctx = default_ctx();
  hipStream_t st = nullptr;   // stream the memory is used on (handed to the allocator)
  std::vector<std::pair<void*, uint64_t>> ptrs;
  uint64_t bytes = 0;
  std::string why;            // reason of the last failed allocation
  DevMem() = default;
  explicit DevMem(std::shared_ptr<CtxState> c, hipStream_t s = nullptr) : ctx(std::move(c)), st(s) {}
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() { reset(); }
  void* raw(uint64_t nbytes) {
    if (!ctx->reserve(nbytes, &why)) return nullptr;
    void* p = nullptr;
    if (ctx->alloc) {
      p = ctx->alloc((size_t)nbytes, (void*)st, ctx->user);
    } else if (hipMalloc(&p, nbytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (!p) {
      if (why.empty()) why = "device allocation failed";
      ctx->unreserve(nbytes);
      return nullptr;
    }
    ptrs.emplace_back(p, nbytes);
    bytes += nbytes;
    return p;
  }
  template <class T>
  T* alloc(size_t n) {
    return static_cast<T*>(raw((uint64_t)std::max<size_t>(n, 1) * sizeof(T)));
  }
  void give_back(void* p, uint64_t nbytes) {
    if (ctx->free_)
      ctx->free_(p, ctx->user);
    else
      hipFree(p);
    ctx->unreserve(nbytes);
  }
  // Memory still used by queued kernels must not go back to a caching
  // allocator: the device is drained first (hipFree waits by itself).
  void drain() {
    if (ctx->free_ && !ptrs.empty()) hipDeviceSynchronize();
  }
  void reset() {
    drain();
    for (auto& q : ptrs) give_back(q.first, q.second);
    ptrs.clear();
    bytes = 0;
  }
  void release(void* p) {
    auto it = std::find_if(ptrs.begin(), ptrs.end(), [&](const std::pair<void*, uint64_t>& q) { return q.first == p; });
    if (it != ptrs.end()) {
      drain();
      give_back(it->first, it->second);
      bytes -= it->second;
      ptrs.erase(it);
    }
  }
};

// bytes of one DevMem allocation of n elements of T (as DevMem::alloc takes)
template <class T>
uint64_t nbytes_of(size_t n) {
  return (uint64_t)std::max<size_t>(n, 1) * sizeof(T);
}

}  // namespace mxw

using namespace mxw;

struct mxw_ctx {
  std::shared_ptr<CtxState> S;
};

static std::shared_ptr<CtxState> ctx_of(mxw_ctx* c) { return c ? c->S : default_ctx(); }

// Host layout plus its device mirror (geometry, numbering, subdomain maps and
// the geometric face matrices), shared by every problem built on it.
struct LayoutShared {
  Layout L;
  std::mutex mu;
  bool on_device = false;
  int device = -1;
  DevMem mem;
  double* xyz = nullptr;
  int* tets = nullptr;
  int* tet_dofs = nullptr;
  Term *phi = nullptr, *curl = nullptr, *fphi = nullptr;
  double* BF = nullptr;
  int *ft_vert = nullptr, *ft_dofs = nullptr;
  int64_t* rowptr = nullptr;
  int* cols = nullptr;
  int* dof_ent = nullptr;
  int64_t *ent_tet_ptr = nullptr, *ent_imp_ptr = nullptr;
  int *ent_tets = nullptr, *ent_imps = nullptr;
  int *imp_ft = nullptr, *imp_opp = nullptr;
  double *gx = nullptr, *gw = nullptr;
  int nq = 0;
  int64_t *foff = nullptr, *poff = nullptr, *sub_tet_ptr = nullptr, *sub_face_ptr = nullptr;
  int *nsz = nullptr, *lds = nullptr, *sub_dofs = nullptr, *sub_tets = nullptr, *sub_lmap = nullptr;
  int *sub_face_ft = nullptr, *sub_face_lmap = nullptr, *order = nullptr;
  uint8_t* pou = nullptr;
  int64_t *gall_ptr = nullptr, *gall_pos = nullptr;
  uint64_t factor_elems = 0;
  std::vector<int64_t> h_foff;
  std::vector<int> h_lds, h_order;
  std::vector<int> h_imp_opp;
};

struct mxw_layout {
  std::shared_ptr<LayoutShared> S;
};

struct KrylovWork {
  int nrhs = 0, m = 0;
  int64_t ndof = 0;
  DevMem mem;
  double2 *V = nullptr, *Z = nullptr, *W = nullptr, *X = nullptr, *Rv = nullptr, *YS = nullptr;
  double2 *h1 = nullptr, *h2 = nullptr, *part = nullptr, *H = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
  double *cs = nullptr, *hn = nullptr, *w0 = nullptr, *npart = nullptr, *est = nullptr, *beta = nullptr;
  int *active = nullptr, *jd = nullptr;
  void* xbuf = nullptr;     // multi-column local solve workspace
  double* host = nullptr;   // pinned: est, hn, w0 for every column
  std::vector<hipGraphExec_t> graphs;   // captured Arnoldi step per index j
  int graph_nrhs = 0;                   // column count the graphs were captured for
  hipStream_t cap = nullptr;            // private capture stream
  void drop_graphs() {
    for (auto& e : graphs)
      if (e) hipGraphExecDestroy(e);
    graphs.clear();
    graph_nrhs = 0;
  }
  ~KrylovWork() {
    drop_graphs();
    if (cap) hipStreamDestroy(cap);
  }
  std::vector<std::vector<double>> history;   // per column: |g_{j+1}| / ||b|| of every step
};

// Block GMRES workspace (one shared Krylov space for p right-hand sides); the
// bases V, Z and the vectors W, R of KrylovWork are reused with block layout
// (vector i*p + c of the basis is column c of block i).
struct BlockWork {
  int p = 0, m = 0, nparts = 0;
  int64_t ndof = 0;
  DevMem mem;
  double2 *H1 = nullptr, *H2 = nullptr, *Hc = nullptr, *part = nullptr, *G = nullptr, *G0 = nullptr, *R1 = nullptr,
          *R1i = nullptr, *R2 = nullptr, *R2i = nullptr, *S = nullptr, *T = nullptr, *Rls = nullptr, *E = nullptr,
          *Y = nullptr;
  double2* Xi = nullptr;   // interleaved copy of a block for the product with A (p >= 16)
  double2* Vi = nullptr;   // interleaved copy of a basis block for the local solves' gather (p >= 16)
  double* est = nullptr;
  int* info = nullptr;   // [0] rank loss, [1] second Gram-Schmidt pass needed
  int64_t reorth = 0;    // second passes in the last solve
  int64_t deflated = 0;  // block steps with a floor pivot in the Cholesky QR
  std::vector<hipGraphExec_t> graphs;   // captured block Arnoldi step per index j
  void drop_graphs() {
    for (auto& e : graphs)
      if (e) hipGraphExecDestroy(e);
    graphs.clear();
  }
  ~BlockWork() { drop_graphs(); }
};

// Krylov recycling (GCRO-DR) state, kept across solves: the basis array
// VC = [C | V_0 .. V_steps] (C: the dim recycled vectors), U and Ubar =
// M^{-1} U beside it, and the small cycle matrices.
struct RecycleWork {
  int k = 0, m = 0, dim = 0;
  int p = 1;            // block width the workspace is sized for (Block GCRO-DR)
  int64_t ndof = 0;
  uint64_t gen = 0;   // operator generation C = A Ubar was made for
  DevMem mem;
  double2 *VC = nullptr, *Zs = nullptr, *U = nullptr, *Ub = nullptr, *Ut = nullptr, *Ubt = nullptr, *Ct = nullptr;
  double2 *W = nullptr, *R = nullptr, *YS = nullptr;
  double2 *h1 = nullptr, *h2 = nullptr, *part = nullptr, *H = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
  double2 *t = nullptr, *G = nullptr, *WVg = nullptr, *UU = nullptr, *Mc = nullptr, *Mu = nullptr, *mu = nullptr;
  double *cs = nullptr, *w0 = nullptr, *hn = nullptr, *npart = nullptr, *est = nullptr, *beta = nullptr;
  int *jd = nullptr, *info = nullptr, *kd = nullptr;
  void* xbuf = nullptr;
  double* host = nullptr;   // pinned
  BlockWork bw;             // Gram products and Cholesky QR
  // block cycles: coefficients against C of the two passes, the recycled
  // part of the update, and the block least-squares state
  double2 *B1 = nullptr, *B2 = nullptr, *Tb = nullptr;
  double *npb = nullptr, *bnb = nullptr;   // column norms of a block: partials, results
  BlockWork bb;
  std::vector<double> history;
  int64_t refreshes = 0, deflations = 0, failures = 0;
  ~RecycleWork() {
    if (host) hipHostFree(host);
  }
};

struct mxw_problem {
  mxw_problem(std::shared_ptr<LayoutShared> s, std::shared_ptr<CtxState> c, hipStream_t st)
      : S(std::move(s)), L(S->L), ctx(c), mem(c, st) {
    kw.mem.ctx = bw.mem.ctx = rw.mem.ctx = rw.bw.mem.ctx = rw.bb.mem.ctx = c;
  }
  std::shared_ptr<LayoutShared> S;
  const Layout& L;
  std::shared_ptr<CtxState> ctx;
  std::mutex run;          // held by a solve (solves on one problem run one after another)
  int device = 0;
  int variant = MXW_PREC_ORAS;
  double k0 = 0.0;
  DevMem mem;
  // per-problem (medium dependent) device data
  double* eps = nullptr;
  double *imp_beta = nullptr, *imp_eps = nullptr, *sub_face_coef = nullptr;
  double2* AT = nullptr;
  double2* vals = nullptr;
  int *perm = nullptr, *info = nullptr;
  void* F = nullptr;
  void* lu_scratch = nullptr;
  // views of the shared layout mirror
  double* xyz = nullptr;
  int* tets = nullptr;
  int* tet_dofs = nullptr;
  Term *phi = nullptr, *curl = nullptr, *fphi = nullptr;
  double* BF = nullptr;
  int *ft_vert = nullptr, *ft_dofs = nullptr;
  int64_t* rowptr = nullptr;
  int* cols = nullptr;
  int* dof_ent = nullptr;
  int64_t *ent_tet_ptr = nullptr, *ent_imp_ptr = nullptr;
  int *ent_tets = nullptr, *ent_imps = nullptr;
  int *imp_ft = nullptr, *imp_opp = nullptr;
  double *gx = nullptr, *gw = nullptr;
  int nq = 0;
  int64_t *foff = nullptr, *poff = nullptr, *sub_tet_ptr = nullptr, *sub_face_ptr = nullptr;
  int *nsz = nullptr, *lds = nullptr, *sub_dofs = nullptr, *sub_tets = nullptr, *sub_lmap = nullptr;
  int *sub_face_ft = nullptr, *sub_face_lmap = nullptr, *order = nullptr;
  uint8_t* pou = nullptr;
  int64_t *gall_ptr = nullptr, *gall_pos = nullptr;
  uint64_t factor_elems = 0;
  bool factored = false;
  bool mixed = false;
  int spmv_group = 16;
  int multi_ku = 8;       // k slice width of the multi-column local solve (tunable)
  int lu_ku = 8;          // k slice width of the LU's block-column update (tunable in FP32)
  int multi_rows = 64;    // rows per pass of the multi-column local solve (64, or 128 in FP32; tunable)
  uint64_t op_gen = 0;    // bumped whenever A or M changes (recycled spaces go stale)
  // factor residency per subdomain (assemble_medium)
  int* sub_list = nullptr;             // device: subdomains to re-factorise
  int* lu_counter = nullptr;           // device: work counter of the persistent LU launch
  bool lu_persistent = false;          // LU launch: persistent queue (tunable) or one workgroup per subdomain
  std::vector<uint64_t> sub_hash;      // local-data hash each subdomain's factors were made for
  bool hash_valid = false;             // the factors match sub_hash (no failed or deferred factorisation)
  int64_t refactor_last = 0, refactor_total = 0, kept_total = 0, medium_updates = 0;
  KrylovWork kw;
  BlockWork bw;
  RecycleWork rw;
};

namespace {

mxw_status dev_fail(const char* what, hipError_t e) {
  std::ostringstream os;
  os << what << ": " << hipGetErrorString(e);
  set_error(os.str());
  return MXW_EDEVICE;
}

#define HIP_CHECK(x)                                  \
  do {                                                \
    hipError_t e_ = (x);                              \
    if (e_ != hipSuccess) return dev_fail(#x, e_);    \
  } while (0)

template <class T>
mxw_status upload(DevMem& mem, T*& dst, const std::vector<T>& src, hipStream_t st) {
  dst = mem.alloc<T>(src.size());
  if (!dst) {
    set_error(mem.why);
    return MXW_ENOMEM;
  }
  if (!src.empty()) HIP_CHECK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return MXW_OK;
}

#define TRY(x)                    \
  do {                            \
    mxw_status s_ = (x);          \
    if (s_ != MXW_OK) return s_;  \
  } while (0)

int64_t round_ld(int64_t n) { return (n + 7) / 8 * 8; }

// Gauss-Legendre nodes and weights on [0,1] (Newton iteration on P_n).
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? z : p1;
      double pm = (n == 1) ? 1.0 : p0;
      double dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double pn = (n == 1) ? z : p1;
    double pm = (n == 1) ? 1.0 : p0;
    double dp = n * (z * pn - pm) / (z * z - 1.0);
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);   // = 0.5 * 2/((1-z^2) P'^2)
  }
}

// ---- exact device footprints: each function lists the allocations of the
// code it sizes, in the same order and with the same element counts

// the layout's device copy (ensure_device_layout)
uint64_t mirror_bytes(const Layout& L) {
  uint64_t b = 0;
  b += nbytes_of<double>(L.xyz.size()) + nbytes_of<int>(L.tets.size()) + nbytes_of<int>(L.tet_dofs.size());
  b += nbytes_of<Term>(L.basis.phi.size()) + nbytes_of<Term>(L.basis.curl.size()) +
       nbytes_of<Term>(L.basis.fphi.size());
  b += nbytes_of<int>(L.ft_vert.size()) + nbytes_of<int>(L.ft_dofs.size());
  b += nbytes_of<int64_t>(L.rowptr.size()) + nbytes_of<int>(L.cols.size()) + nbytes_of<int>(L.dof_ent.size());
  b += nbytes_of<int64_t>(L.ent_tet_ptr.size()) + nbytes_of<int>(L.ent_tets.size());
  b += nbytes_of<int64_t>(L.ent_imp_ptr.size()) + nbytes_of<int>(L.ent_imps.size());
  b += nbytes_of<int>(L.imp_ft.size()) + nbytes_of<int>(L.imp_ft.size());    // imp_ft, imp_opp
  b += 2 * nbytes_of<double>(L.r + 3);                                         // gx, gw
  b += nbytes_of<int64_t>(L.n_sub) + nbytes_of<int64_t>(L.n_sub + 1);          // foff, poff
  b += 3 * nbytes_of<int>(L.n_sub);                                             // nsz, lds, order
  b += nbytes_of<int>(L.sub_dofs.size()) + nbytes_of<uint8_t>(L.sub_pou.size());
  b += nbytes_of<int64_t>(L.sub_tet_ptr.size()) + nbytes_of<int>(L.sub_tets.size()) +
       nbytes_of<int>(L.sub_lmap.size());
  b += nbytes_of<int64_t>(L.sub_face_ptr.size()) + nbytes_of<int>(L.sub_face_ft.size()) +
       nbytes_of<int>(L.sub_face_lmap.size());
  b += nbytes_of<int64_t>(L.ndof + 1) + nbytes_of<int64_t>(L.sub_dofs.size());  // gall_ptr, gall_pos
  b += nbytes_of<double>(L.ft_face.size() * (size_t)L.basis.nfloc * L.basis.nfloc);   // BF
  return b;
}

uint64_t factor_elems_of(const Layout& L) {
  uint64_t e = 0;
  for (int s = 0; s < L.n_sub; ++s) {
    const int64_t n = L.sub_dof_ptr[s + 1] - L.sub_dof_ptr[s];
    e += 2 * (uint64_t)round_ld(n) * n;
  }
  return e;
}

// one problem's operator, element matrices and factors (create_problem)
uint64_t problem_bytes(const Layout& L, int precision) {
  const size_t rsz = precision == MXW_MIXED ? 4 : 8;
  const int nloc = L.basis.nloc;
  uint64_t b = 0;
  b += nbytes_of<double>(2 * L.nt) + nbytes_of<double>(L.imp_tet.size()) + nbytes_of<double>(2 * L.imp_tet.size());
  b += nbytes_of<double>(L.sub_face_tet.size());
  b += nbytes_of<int>(L.sum_ns) + nbytes_of<int>(L.n_sub);                     // perm, info
  b += nbytes_of<unsigned char>(factor_elems_of(L) * rsz);                      // F
  b += nbytes_of<unsigned char>((size_t)L.sum_ns * 2 * kLuNB * rsz);            // LU block-column scratch
  b += nbytes_of<double2>((size_t)L.nt * nloc * nloc);                           // AT
  b += nbytes_of<double2>(L.cols.size());                                       // CSR values
  b += nbytes_of<int>(L.n_sub);                                                 // subdomain list
  b += nbytes_of<int>(1);                                                       // LU work counter
  return b;
}

// variants whose prolongation gathers every local solution of an unknown
// (OAS: D_s = I; ORAS_MULT: weights by multiplicity) instead of the owner's
bool gathered(int variant) { return variant == MXW_PREC_OAS || variant == MXW_PREC_ORAS_MULT; }

// the Krylov workspace for nrhs columns (ensure_krylov)
uint64_t krylov_bytes(const Layout& L, int nrhs, int m, int variant, bool mixed) {
  const int64_t n = L.ndof;
  const int maxv = m + 1;
  const int nblk = red_blocks(n);
  uint64_t b = 0;
  b += nbytes_of<double2>((size_t)nrhs * maxv * n) + nbytes_of<double2>((size_t)nrhs * m * n);   // V, Z
  b += 3 * nbytes_of<double2>((size_t)nrhs * n);                                                // W, X, Rv
  if (gathered(variant)) b += nbytes_of<double2>((size_t)nrhs * L.sum_ns);                     // YS
  b += 2 * nbytes_of<double2>((size_t)nrhs * maxv);                                            // h1, h2
  b += nbytes_of<double2>((size_t)nrhs * nblk * maxv);                                          // part
  b += nbytes_of<double2>((size_t)nrhs * maxv * m);                                             // H
  b += nbytes_of<double2>((size_t)nrhs * maxv) + nbytes_of<double2>((size_t)nrhs * (maxv + 1));  // sn, g
  b += nbytes_of<double2>((size_t)nrhs * maxv);                                                 // y
  b += nbytes_of<double>((size_t)nrhs * maxv);                                                  // cs
  b += 2 * nbytes_of<double>(nrhs) + nbytes_of<double>((size_t)nrhs * nblk) + 2 * nbytes_of<double>(nrhs);
  b += 2 * nbytes_of<int>(nrhs);                                                                // active, jd
  if (nrhs >= 2 && !gathered(variant)) {
    const int nchunk = (nrhs + multi_chunk_cols() - 1) / multi_chunk_cols();
    b += nbytes_of<unsigned char>((size_t)nchunk * 2 * L.sum_ns * multi_chunk_cols() * (mixed ? 4 : 8));
  }
  return b;
}

constexpr int kMaxGramParts = 128;   // split-K partial products of a Gram matrix

// blocks of at least this many columns multiply A through an interleaved copy
constexpr int kIlMinCols = 16;

// the block GMRES workspace (ensure_block_ws)
uint64_t block_bytes(int64_t n, int p, int m) {
  const int64_t Q = (int64_t)(m + 1) * p;
  uint64_t b = 0;
  b += 3 * nbytes_of<double2>(Q * p);                                  // H1, H2, Hc
  b += nbytes_of<double2>((size_t)kMaxGramParts * Q * p);              // part
  b += 7 * nbytes_of<double2>((size_t)p * p);                          // G, G0, R1, R1i, R2, R2i, S
  b += nbytes_of<double2>((size_t)m * 4 * p * p);                      // T
  b += nbytes_of<double2>((size_t)m * p * m * p);                      // Rls
  b += nbytes_of<double2>(Q * p) + nbytes_of<double2>((size_t)m * p * p);   // E, Y
  b += nbytes_of<double>(p) + nbytes_of<int>(2);                       // est, info
  if (p >= kIlMinCols) b += 2 * nbytes_of<double2>((size_t)n * interleaved_cols());   // Xi, Vi
  return b;
}

// temporaries of one mxw_solve call: right-hand sides, solution staging for
// a host output, face integrals of plane-wave / port sources
uint64_t solve_temp_bytes(const Layout& L, int nrhs) {
  return 2 * nbytes_of<double2>((size_t)L.ndof * nrhs) +
         nbytes_of<double2>(std::max<size_t>(1, L.imp_ft.size() * (size_t)L.basis.nfloc));
}

uint64_t footprint_bytes(const Layout& L, int precision, int variant, int nrhs, int m, int krylov, bool with_mirror) {
  nrhs = std::max(nrhs, 1);
  uint64_t b = problem_bytes(L, precision) + krylov_bytes(L, nrhs, m, variant, precision == MXW_MIXED) +
               solve_temp_bytes(L, nrhs);
  if (krylov == MXW_KRYLOV_BLOCK) b += block_bytes(L.ndof, nrhs, m);
  if (with_mirror) b += mirror_bytes(L);
  return b;
}


mxw_status ensure_krylov(mxw_problem* P, int nrhs, int m) {
  KrylovWork& k = P->kw;
  if (k.nrhs >= nrhs && k.m == m && k.ndof == P->L.ndof && k.V) return MXW_OK;
  k.drop_graphs();
  P->bw.drop_graphs();   // block steps captured with the old bases
  k.mem.reset();
  if (k.host) {
    hipHostFree(k.host);
    k.host = nullptr;
  }
  const int64_t n = P->L.ndof;
  const int maxv = m + 1;
  const int nblk = red_blocks(n);
  k.nrhs = nrhs;
  k.m = m;
  k.ndof = n;
  k.V = k.mem.alloc<double2>((size_t)nrhs * maxv * n);
  k.Z = k.mem.alloc<double2>((size_t)nrhs * m * n);
  k.W = k.mem.alloc<double2>((size_t)nrhs * n);
  k.X = k.mem.alloc<double2>((size_t)nrhs * n);
  k.Rv = k.mem.alloc<double2>((size_t)nrhs * n);
  k.YS = gathered(P->variant) ? k.mem.alloc<double2>((size_t)nrhs * P->L.sum_ns) : nullptr;
  k.h1 = k.mem.alloc<double2>((size_t)nrhs * maxv);
  k.h2 = k.mem.alloc<double2>((size_t)nrhs * maxv);
  k.part = k.mem.alloc<double2>((size_t)nrhs * nblk * maxv);
  k.H = k.mem.alloc<double2>((size_t)nrhs * maxv * m);
  k.sn = k.mem.alloc<double2>((size_t)nrhs * maxv);
  k.g = k.mem.alloc<double2>((size_t)nrhs * (maxv + 1));
  k.y = k.mem.alloc<double2>((size_t)nrhs * maxv);
  k.cs = k.mem.alloc<double>((size_t)nrhs * maxv);
  k.hn = k.mem.alloc<double>(nrhs);
  k.w0 = k.mem.alloc<double>(nrhs);
  k.npart = k.mem.alloc<double>((size_t)nrhs * nblk);
  k.est = k.mem.alloc<double>(nrhs);
  k.beta = k.mem.alloc<double>(nrhs);
  k.active = k.mem.alloc<int>(nrhs);
  k.jd = k.mem.alloc<int>(nrhs);
  if (!k.V || !k.Z || !k.W || !k.X || !k.Rv || !k.h1 || !k.h2 || !k.part || !k.H || !k.sn || !k.g || !k.y ||
      !k.cs || !k.hn || !k.w0 || !k.npart || !k.est || !k.beta || !k.active || !k.jd ||
      (gathered(P->variant) && !k.YS)) {
    k.V = nullptr;
    set_error("Krylov workspace: " + k.mem.why);
    return MXW_ENOMEM;
  }
  k.xbuf = nullptr;
  if (nrhs >= 2 && !gathered(P->variant)) {
    const int nchunk = (nrhs + multi_chunk_cols() - 1) / multi_chunk_cols();
    k.xbuf = k.mem.alloc<unsigned char>((size_t)nchunk * 2 * P->L.sum_ns * multi_chunk_cols() * (P->mixed ? 4 : 8));
    if (!k.xbuf) {
      k.V = nullptr;
      set_error("Krylov workspace (multi-column local solve): " + k.mem.why);
      return MXW_ENOMEM;
    }
  }
  if (hipHostMalloc((void**)&k.host, sizeof(double) * 4 * nrhs) != hipSuccess) {
    set_error("pinned host allocation failed");
    return MXW_ENOMEM;
  }
  return MXW_OK;
}

// z = M^{-1} v for ncol columns (device, stride ndof)
// vil (optional): the interleaved copy of v, gathered by the multi-column
// solves instead of v (at most interleaved_cols() columns)
void apply_prec_dev(mxw_problem* P, hipStream_t st, const double2* v, int64_t vstride, double2* z, int64_t zstride,
                    int ncol, const int* active, double2* ys, void* xbuf = nullptr, const double2* vil = nullptr) {
  if (xbuf && ncol >= 2 && !gathered(P->variant)) {
    ScopedKernelTimer tm("local_solve_multi");
    LocalSolveArgs a{P->L.n_sub, (int)P->L.max_ns, P->foff, P->nsz, P->lds, P->perm, P->poff, P->sub_dofs, P->pou,
                     P->order, vil};
    if (P->mixed)
      launch_local_solve_multi<float>(st, a, (const float*)P->F, v, vstride, z, zstride, (float*)xbuf, P->L.sum_ns,
                                      ncol, active, P->multi_ku, P->multi_rows);
    else
      launch_local_solve_multi<double>(st, a, (const double*)P->F, v, vstride, z, zstride, (double*)xbuf,
                                       P->L.sum_ns, ncol, active, P->multi_ku, P->multi_rows);
    return;
  }
  ScopedKernelTimer tm("local_solve");
  LocalSolveArgs a{P->L.n_sub, (int)P->L.max_ns, P->foff, P->nsz, P->lds, P->perm, P->poff, P->sub_dofs, P->pou,
                   P->order};
  const int64_t n = P->L.ndof;
  const bool oas = gathered(P->variant);
  if (P->mixed)
    launch_local_solve<float>(st, a, (const float*)P->F, v, vstride, z, zstride, oas ? ys : nullptr, P->L.sum_ns, ncol,
                              active);
  else
    launch_local_solve<double>(st, a, (const double*)P->F, v, vstride, z, zstride, oas ? ys : nullptr, P->L.sum_ns,
                               ncol, active);
  if (oas)
    launch_gather_all(st, n, P->gall_ptr, P->gall_pos, ys, P->L.sum_ns, z, zstride, ncol, active,
                      P->variant == MXW_PREC_ORAS_MULT);
}

void spmv_dev(mxw_problem* P, hipStream_t st, const double2* x, double2* y, const double2* b, int ncol,
              const int* active) {
  ScopedKernelTimer tm("spmv");
  const int64_t n = P->L.ndof;
  launch_spmv(st, P->spmv_group, n, P->rowptr, P->cols, P->vals, x, n, y, n, b, n, ncol, active);
}

// A port source: centre, unit vectors along the wide (u) and narrow (v)
// sides, width a and height b.
struct PortFrame {
  double c[3], u[3], v[3], a, b;
};

mxw_status port_frame(const mxw_source& S, PortFrame& f) {
  const double hw = std::sqrt(S.dir[0] * S.dir[0] + S.dir[1] * S.dir[1] + S.dir[2] * S.dir[2]);
  const double hh = std::sqrt(S.pol_re[0] * S.pol_re[0] + S.pol_re[1] * S.pol_re[1] + S.pol_re[2] * S.pol_re[2]);
  const double dot = S.dir[0] * S.pol_re[0] + S.dir[1] * S.pol_re[1] + S.dir[2] * S.pol_re[2];
  if (S.kind != MXW_SRC_PORT || !(hw > 0) || !(hh > 0) || std::fabs(dot) > 1e-9 * hw * hh) {
    set_error("a port needs non-zero, orthogonal half-width (dir) and half-height (pol_re) vectors");
    return MXW_EINVAL;
  }
  for (int q = 0; q < 3; ++q) {
    f.c[q] = S.pos[q];
    f.u[q] = S.dir[q] / hw;
    f.v[q] = S.pol_re[q] / hh;
  }
  f.a = 2.0 * hw;
  f.b = 2.0 * hh;
  return MXW_OK;
}

mxw_status check_problem(const mxw_problem* P) {
  if (!P) {
    set_error("problem is NULL");
    return MXW_EINVAL;
  }
  return MXW_OK;
}

// list / count: the subdomains to assemble (device ids, largest first);
// nullptr = all of them
// the LU's launch: persistent queue or one workgroup per subdomain
int* lu_queue(mxw_problem* P) { return P->lu_persistent ? P->lu_counter : nullptr; }

template <typename R>
mxw_status build_local_and_factor(mxw_problem* P, hipStream_t st, bool factor, const int* list = nullptr,
                                  int count = -1) {
  const Layout& L = P->L;
  LocalAssembleArgs la{list ? count : L.n_sub, P->foff, P->nsz, P->lds, P->sub_tet_ptr, P->sub_tets, P->sub_lmap,
                       P->AT, L.basis.nloc, P->sub_face_ptr, P->sub_face_ft, P->sub_face_coef, P->sub_face_lmap,
                       P->BF, L.basis.nfloc, list};
  {
    ScopedTimer tm(st, "local_assemble");
    if (P->variant == MXW_PREC_RAS)
      launch_local_from_csr<R>(st, L.n_sub, (R*)P->F, P->foff, P->nsz, P->lds, P->poff, P->sub_dofs, P->rowptr,
                               P->cols, P->vals);
    else
      launch_assemble_local<R>(st, la, (R*)P->F);
  }
  HIP_CHECK(hipGetLastError());
  if (factor) {
    ScopedKernelTimer tm("lu");
    launch_lu<R>(st, L.n_sub, (R*)P->F, P->foff, P->nsz, P->lds, P->perm, P->poff, (R*)P->lu_scratch, P->info,
                 P->order, P->lu_ku, lu_queue(P));
  }
  HIP_CHECK(hipGetLastError());
  return MXW_OK;
}

// list / count: factorise only these subdomains (device ids, largest first);
// nullptr = all
mxw_status factor_impl(mxw_problem* P, hipStream_t st, const int* list = nullptr, int count = -1) {
  if (P->factored) return MXW_OK;
  const int nf = list ? count : P->L.n_sub;
  const int* ord = list ? list : P->order;
  if (P->mixed) {
    ScopedKernelTimer tm("lu");
    launch_lu<float>(st, nf, (float*)P->F, P->foff, P->nsz, P->lds, P->perm, P->poff, (float*)P->lu_scratch,
                     P->info, ord, P->lu_ku, lu_queue(P));
  } else {
    ScopedKernelTimer tm("lu");
    launch_lu<double>(st, nf, (double*)P->F, P->foff, P->nsz, P->lds, P->perm, P->poff, (double*)P->lu_scratch,
                      P->info, ord, P->lu_ku, lu_queue(P));
  }
  HIP_CHECK(hipGetLastError());
  std::vector<int> info(P->L.n_sub);
  HIP_CHECK(hipMemcpyAsync(info.data(), P->info, sizeof(int) * info.size(), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  P->factored = true;
  ++P->op_gen;
  P->hash_valid = true;
  for (int s = 0; s < P->L.n_sub; ++s)
    if (info[s] != 0) {
      P->hash_valid = false;   // the next medium factorises every subdomain again
      std::ostringstream os;
      os << "zero pivot in the LU of subdomain " << s << " at column " << info[s] - 1;
      set_error(os.str());
      return MXW_ESINGULAR;
    }
  return MXW_OK;
}

}  // namespace

extern "C" {

const char* mxw_last_error(void) { return g_err.c_str(); }

mxw_status mxw_layout_create(const mxw_problem_desc* desc, mxw_layout** out) {
  if (!out) {
    set_error("out is NULL");
    return MXW_EINVAL;
  }
  *out = nullptr;
  std::unique_ptr<mxw_layout> l(new (std::nothrow) mxw_layout());
  if (!l) {
    set_error("host allocation failed");
    return MXW_ENOMEM;
  }
  try {
    l->S = std::make_shared<LayoutShared>();
    TRY(build_layout(desc, l->S->L));
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return MXW_ENOMEM;
  }
  *out = l.release();
  return MXW_OK;
}

void mxw_layout_destroy(mxw_layout* layout) {
  if (!layout) return;
  release_timing_events();   // the device mirror may go with the last reference
  delete layout;
}

static void fill_info(const Layout& L, mxw_layout_info* info) {
  info->ndof = L.ndof;
  info->nnz = L.rowptr.empty() ? 0 : L.rowptr.back();
  info->n_sub = L.n_sub;
  info->nloc = L.basis.nloc;
  info->sum_ns = L.sum_ns;
  info->max_ns = L.max_ns;
  info->sum_ns2 = L.sum_ns2;
  info->sum_ns3 = L.sum_ns3;
  info->n_iface = L.n_iface;
  info->n_imp_faces = (int64_t)L.imp_ft.size();
}

mxw_status mxw_layout_get_info(const mxw_layout* layout, mxw_layout_info* info) {
  if (!layout || !info) {
    set_error("NULL argument");
    return MXW_EINVAL;
  }
  fill_info(layout->S->L, info);
  return MXW_OK;
}

mxw_status mxw_export_dofs(const mxw_layout* layout, int8_t* ent_kind, int64_t* ent_id, int16_t* ent_local) {
  if (!layout || !ent_kind || !ent_id || !ent_local) {
    set_error("NULL argument");
    return MXW_EINVAL;
  }
  const Layout& L = layout->S->L;
  std::copy(L.ent_kind.begin(), L.ent_kind.end(), ent_kind);
  std::copy(L.ent_id.begin(), L.ent_id.end(), ent_id);
  std::copy(L.ent_local.begin(), L.ent_local.end(), ent_local);
  return MXW_OK;
}

mxw_status mxw_export_pattern(const mxw_layout* layout, int64_t* rowptr, int32_t* cols) {
  if (!layout || !rowptr || !cols) {
    set_error("NULL argument");
    return MXW_EINVAL;
  }
  const Layout& L = layout->S->L;
  std::copy(L.rowptr.begin(), L.rowptr.end(), rowptr);
  std::copy(L.cols.begin(), L.cols.end(), cols);
  return MXW_OK;
}

mxw_status mxw_export_subdomain(const mxw_layout* layout, int32_t s, int64_t* n_s, int64_t* dofs, uint8_t* pou) {
  if (!layout || !n_s) {
    set_error("NULL argument");
    return MXW_EINVAL;
  }
  const Layout& L = layout->S->L;
  if (s < 0 || s >= L.n_sub) {
    set_error("subdomain id out of range");
    return MXW_EINVAL;
  }
  const int64_t b = L.sub_dof_ptr[s], e = L.sub_dof_ptr[s + 1];
  *n_s = e - b;
  if (dofs)
    for (int64_t q = b; q < e; ++q) dofs[q - b] = L.sub_dofs[q];
  if (pou) std::copy(L.sub_pou.begin() + b, L.sub_pou.begin() + e, pou);
  return MXW_OK;
}

mxw_status mxw_layout_footprint(const mxw_layout* layout, int32_t precision, int32_t prec_variant, int32_t nrhs,
                                const mxw_solve_opts* opts, int32_t with_layout_copy, uint64_t* bytes) {
  if (!layout || !bytes || nrhs < 0 || (precision != MXW_FP64 && precision != MXW_MIXED) || prec_variant < 0 ||
      prec_variant > MXW_PREC_ORAS_MULT || (opts && (opts->restart < 1 || opts->restart > 200))) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  const int m = opts ? opts->restart : 50;
  const int krylov = opts ? opts->krylov : MXW_KRYLOV_PSEUDOBLOCK;
  *bytes = footprint_bytes(layout->S->L, precision, prec_variant, nrhs, m, krylov, with_layout_copy != 0);
  return MXW_OK;
}

mxw_status mxw_footprint(const mxw_problem_desc* desc, int32_t nrhs, const mxw_solve_opts* opts, uint64_t* bytes) {
  if (!desc || !bytes) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  mxw_layout* l = nullptr;
  TRY(mxw_layout_create(desc, &l));
  const mxw_status st = mxw_layout_footprint(l, desc->precision, desc->prec_variant, nrhs, opts, 1, bytes);
  mxw_layout_destroy(l);
  return st;
}

mxw_status mxw_ctx_create(int32_t device, uint64_t hbm_budget, mxw_alloc_fn alloc, mxw_free_fn free_, void* user,
                          mxw_ctx** out) {
  if (!out || (!alloc) != (!free_)) {
    set_error("out is NULL, or only one of alloc / free_ given");
    return MXW_EINVAL;
  }
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    set_error("no such device");
    return MXW_EINVAL;
  }
  std::unique_ptr<mxw_ctx> c(new (std::nothrow) mxw_ctx());
  if (!c) {
    set_error("host allocation failed");
    return MXW_ENOMEM;
  }
  c->S = std::make_shared<CtxState>();
  c->S->device = device;
  c->S->budget = hbm_budget;
  c->S->alloc = alloc;
  c->S->free_ = free_;
  c->S->user = user;
  *out = c.release();
  return MXW_OK;
}

mxw_status mxw_ctx_destroy(mxw_ctx* ctx) {
  if (!ctx) return MXW_OK;
  {
    std::lock_guard<std::mutex> lk(ctx->S->mu);
    if (ctx->S->live > 0) {
      std::ostringstream os;
      os << "context still holds " << ctx->S->live << " device allocations (" << ctx->S->in_use << " bytes)";
      set_error(os.str());
      return MXW_EBUSY;
    }
  }
  delete ctx;
  return MXW_OK;
}

mxw_status mxw_ctx_usage(mxw_ctx* ctx, uint64_t* in_use, uint64_t* peak, int64_t* live, int32_t reset_peak) {
  CtxState& c = ctx ? *ctx->S : *default_ctx();
  std::lock_guard<std::mutex> lk(c.mu);
  if (in_use) *in_use = c.in_use;
  if (peak) *peak = c.peak;
  if (live) *live = c.live;
  if (reset_peak) c.peak = c.in_use;
  return MXW_OK;
}

}  // extern "C"

namespace {

// Device mirror of a layout: uploaded once, then shared.
mxw_status ensure_device_layout(LayoutShared& S, const std::shared_ptr<CtxState>& ctx, hipStream_t st) {
  std::lock_guard<std::mutex> lk(S.mu);
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  if (S.on_device) {
    if (dev != S.device) {
      set_error("the layout's device data live on another device");
      return MXW_EINVAL;
    }
    return MXW_OK;
  }
  const Layout& L = S.L;
  DevMem& M = S.mem;
  M.reset();          // a failed earlier attempt may have left a part
  M.ctx = ctx;
  M.st = st;
  TRY(upload(M, S.xyz, L.xyz, st));
  TRY(upload(M, S.tets, L.tets, st));
  TRY(upload(M, S.tet_dofs, L.tet_dofs, st));
  TRY(upload(M, S.phi, L.basis.phi, st));
  TRY(upload(M, S.curl, L.basis.curl, st));
  TRY(upload(M, S.fphi, L.basis.fphi, st));
  TRY(upload(M, S.ft_vert, L.ft_vert, st));
  TRY(upload(M, S.ft_dofs, L.ft_dofs, st));
  TRY(upload(M, S.rowptr, L.rowptr, st));
  TRY(upload(M, S.cols, L.cols, st));
  TRY(upload(M, S.dof_ent, L.dof_ent, st));
  TRY(upload(M, S.ent_tet_ptr, L.ent_tet_ptr, st));
  TRY(upload(M, S.ent_tets, L.ent_tets, st));
  TRY(upload(M, S.ent_imp_ptr, L.ent_imp_ptr, st));
  TRY(upload(M, S.ent_imps, L.ent_imps, st));
  TRY(upload(M, S.imp_ft, L.imp_ft, st));
  S.h_imp_opp.resize(L.imp_ft.size());
  for (size_t q = 0; q < L.imp_ft.size(); ++q) {
    const int32_t f = L.ft_face[L.imp_ft[q]];
    const int32_t t = L.imp_tet[q];
    const auto& fv = L.faces[f];
    int o = -1;
    for (int c = 0; c < 4; ++c) {
      const int32_t v = L.tets[4 * (int64_t)t + c];
      if (v != fv[0] && v != fv[1] && v != fv[2]) o = v;
    }
    S.h_imp_opp[q] = o;
  }
  TRY(upload(M, S.imp_opp, S.h_imp_opp, st));
  {
    std::vector<double> gx, gw;
    S.nq = L.r + 3;
    gauss_legendre01(S.nq, gx, gw);
    TRY(upload(M, S.gx, gx, st));
    TRY(upload(M, S.gw, gw, st));
  }
  {
    std::vector<int64_t> foff(L.n_sub), poff(L.n_sub + 1);
    std::vector<int> nsz(L.n_sub), lds(L.n_sub);
    uint64_t off = 0;
    for (int s = 0; s < L.n_sub; ++s) {
      const int64_t n = L.sub_dof_ptr[s + 1] - L.sub_dof_ptr[s];
      nsz[s] = (int)n;
      lds[s] = (int)round_ld(n);
      foff[s] = (int64_t)off;
      off += 2 * (uint64_t)lds[s] * n;
      poff[s] = L.sub_dof_ptr[s];
    }
    poff[L.n_sub] = L.sub_dof_ptr[L.n_sub];
    S.factor_elems = off;
    S.h_foff = foff;
    S.h_lds = lds;
    std::vector<int> order(L.n_sub);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nsz[a] > nsz[b]; });
    S.h_order = order;
    TRY(upload(M, S.foff, foff, st));
    TRY(upload(M, S.poff, poff, st));
    TRY(upload(M, S.nsz, nsz, st));
    TRY(upload(M, S.lds, lds, st));
    TRY(upload(M, S.order, order, st));
    TRY(upload(M, S.sub_dofs, L.sub_dofs, st));
    TRY(upload(M, S.pou, L.sub_pou, st));
    TRY(upload(M, S.sub_tet_ptr, L.sub_tet_ptr, st));
    TRY(upload(M, S.sub_tets, L.sub_tets, st));
    TRY(upload(M, S.sub_lmap, L.sub_lmap, st));
    TRY(upload(M, S.sub_face_ptr, L.sub_face_ptr, st));
    TRY(upload(M, S.sub_face_ft, L.sub_face_ft, st));
    TRY(upload(M, S.sub_face_lmap, L.sub_face_lmap, st));
    // unknown -> positions in every subdomain's local vector, subdomain order
    std::vector<int64_t> cnt(L.ndof + 1, 0);
    for (int64_t q = 0; q < (int64_t)L.sub_dofs.size(); ++q) cnt[L.sub_dofs[q] + 1]++;
    for (int64_t i = 0; i < L.ndof; ++i) cnt[i + 1] += cnt[i];
    std::vector<int64_t> pos(L.sub_dofs.size()), fill(cnt.begin(), cnt.end() - 1);
    for (int64_t q = 0; q < (int64_t)L.sub_dofs.size(); ++q) pos[fill[L.sub_dofs[q]]++] = q;
    TRY(upload(M, S.gall_ptr, cnt, st));
    TRY(upload(M, S.gall_pos, pos, st));
  }
  const int nfloc = L.basis.nfloc;
  S.BF = M.alloc<double>(L.ft_face.size() * nfloc * nfloc);
  if (!S.BF) {
    set_error("device allocation failed (face matrices)");
    return MXW_ENOMEM;
  }
  {
    ScopedTimer tm(st, "assemble");
    launch_face(st, (int64_t)L.ft_face.size(), S.xyz, S.ft_vert, S.fphi, nfloc, S.BF);
  }
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(st));
  S.device = dev;
  S.on_device = true;
  return MXW_OK;
}

// Everything that depends on the medium, in the problem's existing buffers:
// face coefficients, FP64 element matrices, CSR values, dense A_s and (unless
// deferred) their LU factors.
// Hash of everything a Robin local matrix A_s depends on besides the mesh:
// k0 and the permittivity of every element of Omega_s (its element matrices,
// the impedance and transmission coefficients of its faces), in order.
// FNV-1a over the bytes.
std::vector<uint64_t> local_data_hashes(const Layout& L, const double* eps, double k0) {
  std::vector<uint64_t> h(L.n_sub);
  auto mix = [](uint64_t x, const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t q = 0; q < n; ++q) x = (x ^ c[q]) * 1099511628211ull;
    return x;
  };
  for (int s = 0; s < L.n_sub; ++s) {
    uint64_t x = mix(14695981039346656037ull, &k0, sizeof(k0));
    for (int64_t q = L.sub_tet_ptr[s]; q < L.sub_tet_ptr[s + 1]; ++q)
      x = mix(x, eps + 2 * (int64_t)L.sub_tets[q], 2 * sizeof(double));
    h[s] = x;
  }
  return h;
}

mxw_status assemble_medium(mxw_problem* P, const double* eps, double k0, hipStream_t st, int defer_factor) {
  const Layout& L = P->L;
  const int nloc = L.basis.nloc, nfloc = L.basis.nfloc;
  // factor residency per subdomain: a subdomain whose local data are
  // unchanged keeps its factors (Robin local matrices only: RAS takes A_s
  // from rows of A that reach outside Omega_s)
  std::vector<uint64_t> hash = local_data_hashes(L, eps, k0);
  std::vector<int> changed;
  const bool partial = !defer_factor && P->factored && P->hash_valid && P->variant != MXW_PREC_RAS &&
                       P->sub_hash.size() == hash.size();
  if (partial)
    for (int s : P->S->h_order)   // largest first, as the full launches
      if (hash[s] != P->sub_hash[s]) changed.push_back(s);
  std::vector<double> beta, coef, ie(2 * L.imp_tet.size());
  face_coefficients(L, eps, k0, beta, coef);
  for (size_t q = 0; q < L.imp_tet.size(); ++q) {
    ie[2 * q] = eps[2 * (int64_t)L.imp_tet[q]];
    ie[2 * q + 1] = eps[2 * (int64_t)L.imp_tet[q] + 1];
  }
  HIP_CHECK(hipMemcpyAsync(P->eps, eps, sizeof(double) * 2 * L.nt, hipMemcpyHostToDevice, st));
  if (!beta.empty())
    HIP_CHECK(hipMemcpyAsync(P->imp_beta, beta.data(), sizeof(double) * beta.size(), hipMemcpyHostToDevice, st));
  if (!ie.empty()) HIP_CHECK(hipMemcpyAsync(P->imp_eps, ie.data(), sizeof(double) * ie.size(), hipMemcpyHostToDevice, st));
  if (!coef.empty())
    HIP_CHECK(hipMemcpyAsync(P->sub_face_coef, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice, st));
  P->k0 = k0;
  P->factored = false;
  ++P->op_gen;
  {
    ScopedTimer tm(st, "assemble");
    launch_element(st, L.nt, P->xyz, P->tets, P->eps, P->phi, P->curl, nloc, L.basis.ncurl_max, k0 * k0, P->AT);
    AssembleArgs aa{L.ndof, P->rowptr, P->cols, P->dof_ent, P->ent_tet_ptr, P->ent_tets, P->ent_imp_ptr, P->ent_imps,
                    P->tet_dofs, nloc, P->AT, P->imp_ft, P->imp_beta, P->ft_dofs, nfloc, P->BF, P->vals};
    launch_assemble_rows(st, aa);
  }
  HIP_CHECK(hipGetLastError());
  const int* list = nullptr;
  int count = L.n_sub;
  if (partial) {
    count = (int)changed.size();
    if (count) HIP_CHECK(hipMemcpyAsync(P->sub_list, changed.data(), sizeof(int) * count, hipMemcpyHostToDevice, st));
    list = P->sub_list;
  }
  if (count > 0) {
    if (P->mixed)
      TRY(build_local_and_factor<float>(P, st, false, list, count));
    else
      TRY(build_local_and_factor<double>(P, st, false, list, count));
  }
  HIP_CHECK(hipStreamSynchronize(st));   // the host vectors above go out of scope
  P->sub_hash = hash;
  P->hash_valid = false;
  ++P->medium_updates;
  P->refactor_last = count;
  P->refactor_total += count;
  P->kept_total += L.n_sub - count;
  if (defer_factor) return MXW_OK;
  if (count == 0) {   // every subdomain kept its factors
    P->factored = true;
    P->hash_valid = true;
    return MXW_OK;
  }
  return factor_impl(P, st, list, count);
}

mxw_status create_problem(const std::shared_ptr<CtxState>& ctx, const std::shared_ptr<LayoutShared>& S,
                          const double* eps_in, double k0, int precision, int variant, hipStream_t st,
                          int defer_factor, mxw_problem** out) {
  const Layout& L = S->L;
  if (precision != MXW_FP64 && precision != MXW_MIXED) {
    set_error("unknown precision");
    return MXW_EINVAL;
  }
  if (variant != MXW_PREC_ORAS && variant != MXW_PREC_OAS && variant != MXW_PREC_RAS &&
      variant != MXW_PREC_ORAS_MULT) {
    set_error("unknown preconditioner variant");
    return MXW_EINVAL;
  }
  if (!std::isfinite(k0) || k0 < 0) {
    set_error("k0 must be finite and >= 0");
    return MXW_EINVAL;
  }
  const double* eps = eps_in ? eps_in : L.eps.data();
  for (int64_t q = 0; q < 2 * L.nt; ++q)
    if (!std::isfinite(eps[q])) {
      set_error("non-finite permittivity");
      return MXW_EINVAL;
    }
  const bool mixed = precision == MXW_MIXED;
  if ((uint64_t)L.max_ns * 2 * (mixed ? 4 : 8) > 150 * 1024) {
    std::ostringstream os;
    os << "largest subdomain has " << L.max_ns << " unknowns; the local solve keeps one local vector in LDS "
       << "(at most " << 150 * 1024 / (2 * (mixed ? 4 : 8)) << " unknowns in this precision)";
    set_error(os.str());
    return MXW_EINVAL;
  }
  if (ctx->device >= 0) {   // a context's device (the default context: the current one)
    int cur = 0;
    HIP_CHECK(hipGetDevice(&cur));
    if (cur != ctx->device) HIP_CHECK(hipSetDevice(ctx->device));
  }
  {
    // all or nothing: the operator and factors (and the layout's device copy
    // if this problem builds it) must fit the context's budget
    const uint64_t need = problem_bytes(L, precision) + (S->on_device ? 0 : mirror_bytes(L));
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->budget && ctx->in_use + need > ctx->budget) {
      std::ostringstream os;
      os << "problem needs " << need << " device bytes, " << ctx->in_use << " in use, budget " << ctx->budget;
      set_error(os.str());
      return MXW_ENOMEM;
    }
  }
  TRY(ensure_device_layout(*S, ctx, st));
  std::unique_ptr<mxw_problem> P(new (std::nothrow) mxw_problem(S, ctx, st));
  if (!P) {
    set_error("host allocation failed");
    return MXW_ENOMEM;
  }
  P->device = S->device;
  P->variant = variant;
  P->k0 = k0;
  P->mixed = mixed;
  P->multi_rows = mixed ? 128 : 64;   // measured faster in FP32; in FP64 the LDS of 128 rows halves occupancy
  // persistent LU launch in FP32; in FP64 its loop costs a few spilled registers
  P->lu_persistent = mixed;
  // views of the shared mirror
  P->xyz = S->xyz;
  P->tets = S->tets;
  P->tet_dofs = S->tet_dofs;
  P->phi = S->phi;
  P->curl = S->curl;
  P->fphi = S->fphi;
  P->BF = S->BF;
  P->ft_vert = S->ft_vert;
  P->ft_dofs = S->ft_dofs;
  P->rowptr = S->rowptr;
  P->cols = S->cols;
  P->dof_ent = S->dof_ent;
  P->ent_tet_ptr = S->ent_tet_ptr;
  P->ent_imp_ptr = S->ent_imp_ptr;
  P->ent_tets = S->ent_tets;
  P->ent_imps = S->ent_imps;
  P->imp_ft = S->imp_ft;
  P->imp_opp = S->imp_opp;
  P->gx = S->gx;
  P->gw = S->gw;
  P->nq = S->nq;
  P->foff = S->foff;
  P->poff = S->poff;
  P->sub_tet_ptr = S->sub_tet_ptr;
  P->sub_face_ptr = S->sub_face_ptr;
  P->nsz = S->nsz;
  P->lds = S->lds;
  P->sub_dofs = S->sub_dofs;
  P->sub_tets = S->sub_tets;
  P->sub_lmap = S->sub_lmap;
  P->sub_face_ft = S->sub_face_ft;
  P->sub_face_lmap = S->sub_face_lmap;
  P->order = S->order;
  P->pou = S->pou;
  P->gall_ptr = S->gall_ptr;
  P->gall_pos = S->gall_pos;
  P->factor_elems = S->factor_elems;
  // medium-dependent data
  const int nloc = L.basis.nloc, nfloc = L.basis.nfloc;
  DevMem& M = P->mem;
  P->eps = M.alloc<double>(2 * L.nt);
  P->imp_beta = M.alloc<double>(L.imp_tet.size());
  P->imp_eps = M.alloc<double>(2 * L.imp_tet.size());
  P->sub_face_coef = M.alloc<double>(L.sub_face_tet.size());
  P->perm = M.alloc<int>(L.sum_ns);
  P->info = M.alloc<int>(L.n_sub);
  const size_t rsz = mixed ? 4 : 8;
  P->F = M.alloc<unsigned char>(P->factor_elems * rsz);
  // the LU's row-major copy of the current block column, per subdomain: 2 planes x n_s x 32
  P->lu_scratch = M.alloc<unsigned char>((size_t)L.sum_ns * 2 * kLuNB * rsz);
  P->AT = M.alloc<double2>((size_t)L.nt * nloc * nloc);
  P->vals = M.alloc<double2>(L.cols.size());
  P->sub_list = M.alloc<int>(L.n_sub);
  P->lu_counter = M.alloc<int>(1);
  if (!P->perm || !P->info || !P->F || !P->lu_scratch || !P->AT || !P->vals || !P->eps || !P->imp_beta ||
      !P->imp_eps || !P->sub_face_coef || !P->sub_list || !P->lu_counter) {
    set_error("device allocation failed (factors or element data)");
    return MXW_ENOMEM;
  }
  {
    const size_t dyn = 2 * (size_t)L.max_ns;
    HIP_CHECK(prepare_local_solve(dyn * 8, dyn * 4));
  }
  const int64_t nnz_row = L.ndof ? L.rowptr.back() / L.ndof : 0;
  P->spmv_group = nnz_row <= 12 ? 4 : nnz_row <= 24 ? 8 : nnz_row <= 64 ? 16 : 32;
  mxw_status result = assemble_medium(P.get(), eps, k0, st, defer_factor);
  if (result != MXW_OK && result != MXW_ESINGULAR) return result;
  *out = P.release();
  return result;
}


// ---------------------------------------------------------------------------
// block FGMRES (one Krylov space shared by the p right-hand sides)
// ---------------------------------------------------------------------------
// with_xi: also the interleaved copy of a block for products with A (block
// GMRES with p >= kIlMinCols)
mxw_status ensure_block_ws(BlockWork& b, int64_t n, int p, int m, bool with_xi = false) {
  const bool want_xi = with_xi && p >= kIlMinCols;
  if (b.p == p && b.m == m && b.ndof == n && b.H1 && (b.Xi != nullptr) == want_xi) return MXW_OK;
  b.drop_graphs();
  b.mem.reset();
  b.p = p;
  b.m = m;
  b.ndof = n;
  b.nparts = kMaxGramParts;
  const int64_t Q = (int64_t)(m + 1) * p;
  b.H1 = b.mem.alloc<double2>(Q * p);
  b.H2 = b.mem.alloc<double2>(Q * p);
  b.Hc = b.mem.alloc<double2>(Q * p);
  b.part = b.mem.alloc<double2>((size_t)b.nparts * Q * p);
  b.G = b.mem.alloc<double2>(p * p);
  b.G0 = b.mem.alloc<double2>(p * p);
  b.R1 = b.mem.alloc<double2>(p * p);
  b.R1i = b.mem.alloc<double2>(p * p);
  b.R2 = b.mem.alloc<double2>(p * p);
  b.R2i = b.mem.alloc<double2>(p * p);
  b.S = b.mem.alloc<double2>(p * p);
  b.T = b.mem.alloc<double2>((size_t)m * 4 * p * p);
  b.Rls = b.mem.alloc<double2>((size_t)m * p * m * p);
  b.E = b.mem.alloc<double2>(Q * p);
  b.Y = b.mem.alloc<double2>((size_t)m * p * p);
  b.est = b.mem.alloc<double>(p);
  b.info = b.mem.alloc<int>(2);
  b.Xi = want_xi ? b.mem.alloc<double2>((size_t)n * interleaved_cols()) : nullptr;
  b.Vi = want_xi ? b.mem.alloc<double2>((size_t)n * interleaved_cols()) : nullptr;
  if (!b.H1 || !b.H2 || !b.Hc || !b.part || !b.G || !b.G0 || !b.R1 || !b.R1i || !b.R2 || !b.R2i || !b.S || !b.T || !b.Rls ||
      !b.E || !b.Y || !b.est || !b.info || (want_xi && (!b.Xi || !b.Vi))) {
    b.H1 = nullptr;
    set_error("block Krylov workspace: " + b.mem.why);
    return MXW_ENOMEM;
  }
  return MXW_OK;
}

mxw_status ensure_block(mxw_problem* P, int p, int m) { return ensure_block_ws(P->bw, P->L.ndof, p, m, true); }

// out (Q x p, column-major) = A^H W, A: Q vectors of length n, W: p vectors,
// as split-K partial products summed in a fixed order
mxw_status gram(BlockWork& b, int64_t n, hipStream_t st, const double2* A, int Q, const double2* W, int p,
                double2* out, const int* cond = nullptr) {
  // about 2048 workgroups, within the partial-product buffer (sized for
  // kMaxGramParts parts of the largest Q)
  const int qtiles = (Q + 63) / 64;
  const int cap = (int)std::min<int64_t>(4096, (int64_t)kMaxGramParts * (b.m + 1) * b.p / Q);
  const int want = std::max(1, std::min(cap, 2048 / qtiles));
  launch_bgram(st, A, Q, W, p, n, want, b.part, cond);
  launch_gram_reduce(st, (int64_t)Q * p, bgram_parts(n, want), b.part, out, cond);
  return MXW_OK;
}

mxw_status gram(mxw_problem* P, hipStream_t st, const double2* A, int Q, const double2* W, int p, double2* out,
                const int* cond = nullptr) {
  return gram(P->bw, P->L.ndof, st, A, Q, W, p, out, cond);
}

// C (n x p) = alpha A M + beta C; A: K vectors of length n, M: K x p (ld ldm)
mxw_status tall_gemm(mxw_problem* P, hipStream_t st, const double2* A, int K, const double2* M, int ldm, int p,
                     double alpha, double beta, double2* C, const int* cond = nullptr) {
  launch_bupdate(st, A, K, M, ldm, p, P->L.ndof, alpha, beta, C, C, cond);
  return MXW_OK;
}

// out = in S^{-1} with orthonormal columns (Cholesky QR twice); tmp: n x p.
// have_gram: b.G already holds in^H in.
mxw_status cholqr2(mxw_problem* P, BlockWork& b, hipStream_t st, const double2* in, double2* tmp, double2* out, int p,
                   bool have_gram = false) {
  const int64_t n = P->L.ndof;
  if (!have_gram) TRY(gram(b, n, st, in, p, in, p, b.G));
  launch_chol(st, p, b.G, b.R1, b.R1i, nullptr, nullptr, b.info);
  TRY(tall_gemm(P, st, in, p, b.R1i, p, p, 1.0, 0.0, tmp));
  TRY(gram(b, n, st, tmp, p, tmp, p, b.G));
  launch_chol(st, p, b.G, b.R2, b.R2i, b.R1, b.S, b.info);
  TRY(tall_gemm(P, st, tmp, p, b.R2i, p, p, 1.0, 0.0, out));
  return MXW_OK;
}

// y = A x (b != nullptr: y = b - A x) for the p columns of a block (stride
// ndof): through the interleaved copy from kIlMinCols columns on (the matrix
// read once), else the column-group product
void block_spmv(mxw_problem* P, hipStream_t st, const double2* x, double2* y, const double2* b, int p) {
  const int64_t n = P->L.ndof;
  ScopedKernelTimer tm("spmv");
  if (p >= kIlMinCols && P->bw.Xi)
    launch_spmm_interleaved(st, n, p, P->rowptr, P->cols, P->vals, x, n, P->bw.Xi, y, n, b, n);
  else
    launch_spmv(st, P->spmv_group, n, P->rowptr, P->cols, P->vals, x, n, y, n, b, n, p, nullptr);
}

mxw_status block_solve(mxw_problem* P, int p, const double2* B, const mxw_solve_opts* opts, hipStream_t st,
                       double2* X, int32_t* iters_out, double* relres_out) {
  const int m = opts->restart;
  const int64_t n = P->L.ndof;
  TRY(ensure_krylov(P, p, m));
  TRY(ensure_block(P, p, m));
  KrylovWork& k = P->kw;
  BlockWork& b = P->bw;
  double* hbuf = k.host;
  const int ldE = (m + 1) * p;
  std::vector<double> bnorm(p), relres(p, 1.0);
  k.history.assign(p, std::vector<double>());
  launch_norm(st, n, B, n, k.npart, k.beta, p, nullptr);
  HIP_CHECK(hipMemcpyAsync(hbuf, k.beta, sizeof(double) * p, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  for (int c = 0; c < p; ++c) {
    bnorm[c] = hbuf[c];
    if (!(bnorm[c] > 0)) {
      set_error("block GMRES needs non-zero, independent right-hand sides");
      return MXW_EINVAL;
    }
  }
  HIP_CHECK(hipMemsetAsync(X, 0, sizeof(double2) * n * p, st));
  HIP_CHECK(hipMemcpyAsync(k.Rv, B, sizeof(double2) * n * p, hipMemcpyDeviceToDevice, st));
  b.reorth = 0;
  b.deflated = 0;
  int steps = 0;
  bool conv = false, breakdown = false;
  while (!conv && steps < opts->max_iters && !breakdown) {
    // V_0 S0 = R
    HIP_CHECK(hipMemsetAsync(b.info, 0, sizeof(int), st));
    TRY(cholqr2(P, P->bw, st, k.Rv, k.W, k.V, p));
    launch_set_e(st, p, ldE, b.S, b.E);
    int jd = 0;
    for (int j = 0; j < m; ++j) {
      double2* Vj = k.V + (int64_t)j * p * n;
      double2* Zj = k.Z + (int64_t)j * p * n;
      const int Q = (j + 1) * p;
      // one block Arnoldi step, every decision on the device: block
      // classical Gram-Schmidt, a second pass only where a column lost more
      // than 1 - 1/sqrt(2) of its norm in the first (flag b.info[1], read by
      // the kernels of that pass), Cholesky QR twice, the least-squares update
      auto step = [&](hipStream_t s) -> mxw_status {
        if (b.Vi && !gathered(P->variant)) {   // the local solves gather whole rows of the block
          launch_to_interleaved(s, n, p, Vj, n, b.Vi);
          apply_prec_dev(P, s, Vj, n, Zj, n, p, nullptr, k.YS, k.xbuf, b.Vi);
        } else {
          apply_prec_dev(P, s, Vj, n, Zj, n, p, nullptr, k.YS, k.xbuf);
        }
        block_spmv(P, s, Zj, k.W, nullptr, p);
        TRY(gram(P, s, k.W, p, k.W, p, b.G0));
        TRY(gram(P, s, k.V, Q, k.W, p, b.H1));
        TRY(tall_gemm(P, s, k.V, Q, b.H1, Q, p, -1.0, 1.0, k.W));
        TRY(gram(P, s, k.W, p, k.W, p, b.G));
        launch_reorth_check(s, p, b.G0, b.G, b.info + 1);
        TRY(gram(P, s, k.V, Q, k.W, p, b.H2, b.info + 1));
        TRY(tall_gemm(P, s, k.V, Q, b.H2, Q, p, -1.0, 1.0, k.W, b.info + 1));
        TRY(gram(P, s, k.W, p, k.W, p, b.G, b.info + 1));   // the Gram matrix after the second pass
        // V_{j+1} S = W
        TRY(cholqr2(P, P->bw, s, k.W, k.Rv, k.V + (int64_t)(j + 1) * p * n, p, true));
        launch_bls_step(s, j, p, m, b.H1, b.H2, b.S, b.Hc, b.T, b.Rls, b.E, b.est, b.info + 1);
        return MXW_OK;
      };
      if (opts->use_graph) {
        // the step of index j captured once per workspace and replayed (fixed
        // device addresses, j and Q as constants; the changing state lives in
        // device memory); capture on a private stream
        if ((int)b.graphs.size() < m) b.graphs.resize(m, nullptr);
        if (!b.graphs[j]) {
          if (!k.cap) HIP_CHECK(hipStreamCreateWithFlags(&k.cap, hipStreamNonBlocking));
          hipGraph_t g = nullptr;
          g_capturing = true;
          hipError_t ce = hipStreamBeginCapture(k.cap, hipStreamCaptureModeThreadLocal);
          mxw_status ss = MXW_OK;
          if (ce == hipSuccess) {
            ss = step(k.cap);
            ce = hipStreamEndCapture(k.cap, &g);
          }
          g_capturing = false;
          if (ce != hipSuccess) return dev_fail("graph capture", ce);
          if (ss != MXW_OK) {
            hipGraphDestroy(g);
            return ss;
          }
          const hipError_t ie = hipGraphInstantiate(&b.graphs[j], g, nullptr, nullptr, 0);
          hipGraphDestroy(g);
          if (ie != hipSuccess) {
            b.graphs[j] = nullptr;
            return dev_fail("hipGraphInstantiate", ie);
          }
        }
        HIP_CHECK(hipGraphLaunch(b.graphs[j], st));
      } else {
        TRY(step(st));
      }
      HIP_CHECK(hipGetLastError());
      // the step's one readback: residual estimates and the two flags
      HIP_CHECK(hipMemcpyAsync(hbuf, b.est, sizeof(double) * p, hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipMemcpyAsync(hbuf + p, b.info, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
      ++steps;
      jd = j + 1;
      bool all = true;
      for (int c = 0; c < p; ++c) {
        k.history[c].push_back(hbuf[c] / bnorm[c]);
        if (!(hbuf[c] <= opts->tol * bnorm[c])) all = false;
      }
      int info[2] = {0, 0};
      std::memcpy(info, hbuf + p, 2 * sizeof(int));
      if (info[1]) ++b.reorth;
      if (info[0]) {
        // the new block is numerically rank deficient: the Cholesky QR kept a
        // floor pivot, the direction carries a negligible weight in the least
        // squares and the true residual at the cycle end decides
        ++b.deflated;
        HIP_CHECK(hipMemsetAsync(b.info, 0, sizeof(int), st));
      }
      for (int c = 0; c < p; ++c)
        if (!std::isfinite(hbuf[c])) breakdown = true;
      if (all || breakdown || steps >= opts->max_iters) break;
    }
    // X += Z Y (only with a finite Y: otherwise the last iterate is kept and
    // the solve ends with a breakdown); R = B - A X
    launch_bls_solve(st, jd * p, p, m, b.Rls, b.E, b.Y);
    {
      std::vector<double2> yh((size_t)m * p * p);
      HIP_CHECK(hipMemcpyAsync(yh.data(), b.Y, sizeof(double2) * yh.size(), hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
      bool finite = true;
      for (int c = 0; c < p && finite; ++c)
        for (int r = 0; r < jd * p; ++r) {
          const double2 v = yh[(size_t)c * m * p + r];
          if (!std::isfinite(v.x) || !std::isfinite(v.y)) {
            finite = false;
            break;
          }
        }
      if (!finite) {
        breakdown = true;
        break;
      }
    }
    TRY(tall_gemm(P, st, k.Z, jd * p, b.Y, m * p, p, 1.0, 1.0, X));
    block_spmv(P, st, X, k.Rv, B, p);
    launch_norm(st, n, k.Rv, n, k.npart, k.beta, p, nullptr);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(hbuf, k.beta, sizeof(double) * p, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    conv = true;
    for (int c = 0; c < p; ++c) {
      relres[c] = hbuf[c] / bnorm[c];
      if (!(relres[c] <= opts->tol)) conv = false;
      if (!std::isfinite(relres[c])) breakdown = true;
    }
    if (conv) breakdown = false;
  }
  for (int c = 0; c < p; ++c) {
    if (iters_out) iters_out[c] = steps;
    if (relres_out) relres_out[c] = relres[c];
  }
  if (conv) return MXW_OK;
  if (breakdown) {
    set_error("block Krylov breakdown (non-finite values) before the tolerance");
    return MXW_EBREAKDOWN;
  }
  set_error("max_iters reached before the tolerance");
  return MXW_ENOTCONV;
}


// ---------------------------------------------------------------------------
// Krylov subspace recycling: GCRO-DR over the systems solved on a problem
// (Sec. 6 proposes it for the slowly varying systems of the imaging loop)
// ---------------------------------------------------------------------------
// Buffers whose size follows the block width p (1 for GCRO-DR, p >= 2 for
// Block GCRO-DR): [C, V] (m + p vectors), W, R, the preconditioner's
// staging for max(k, p) columns, the coefficients against C, the column
// norms and the block least-squares state.  A new width keeps the recycled
// space: C moves into the new [C, V].
mxw_status recycle_width(mxw_problem* P, hipStream_t st, int p) {
  RecycleWork& w = P->rw;
  const int64_t n = P->L.ndof;
  const int k = w.k, m = w.m, nblk = red_blocks(n);
  const bool gath = gathered(P->variant);
  const int wide = std::max(k, p);   // columns of a preconditioner application
  std::vector<void*> old = {w.VC, w.W, w.R, w.YS, w.npb, w.bnb, w.B1, w.B2, w.Tb, w.xbuf};
  double2* VC = w.mem.alloc<double2>((size_t)(m + p) * n);
  double2* W = w.mem.alloc<double2>((size_t)p * n);
  double2* R = w.mem.alloc<double2>((size_t)p * n);
  double2* YS = gath ? w.mem.alloc<double2>((size_t)wide * P->L.sum_ns) : nullptr;
  double* npb = w.mem.alloc<double>((size_t)p * nblk);
  double* bnb = w.mem.alloc<double>(p);
  double2* B1 = w.mem.alloc<double2>((size_t)kRecycleMaxK * p);
  double2* B2 = w.mem.alloc<double2>((size_t)kRecycleMaxK * p);
  double2* Tb = w.mem.alloc<double2>((size_t)kRecycleMaxK * p);
  void* xbuf = nullptr;
  bool ok = VC && W && R && (!gath || YS) && npb && bnb && B1 && B2 && Tb;
  if (ok && wide >= 2 && !gath) {
    const int nchunk = (wide + multi_chunk_cols() - 1) / multi_chunk_cols();
    xbuf = w.mem.alloc<unsigned char>((size_t)nchunk * 2 * P->L.sum_ns * multi_chunk_cols() * (P->mixed ? 4 : 8));
    ok = xbuf != nullptr;
  }
  if (!ok) {
    for (void* q : {(void*)VC, (void*)W, (void*)R, (void*)YS, (void*)npb, (void*)bnb, (void*)B1, (void*)B2, (void*)Tb,
                    xbuf})
      if (q) w.mem.release(q);
    set_error("recycling workspace allocation failed");
    return MXW_ENOMEM;
  }
  if (w.VC && w.dim) {
    HIP_CHECK(hipMemcpyAsync(VC, w.VC, sizeof(double2) * w.dim * n, hipMemcpyDeviceToDevice, st));
    HIP_CHECK(hipStreamSynchronize(st));
  }
  for (void* q : old)
    if (q) w.mem.release(q);
  w.VC = VC;
  w.W = W;
  w.R = R;
  w.YS = YS;
  w.npb = npb;
  w.bnb = bnb;
  w.B1 = B1;
  w.B2 = B2;
  w.Tb = Tb;
  w.xbuf = xbuf;
  w.p = p;
  return MXW_OK;
}

// A change of k or m drops the recycled space; a wider block than before
// grows the width-dependent buffers and keeps it (a narrower one uses them
// as they are).
mxw_status ensure_recycle(mxw_problem* P, hipStream_t st, int k, int m, int p = 1) {
  RecycleWork& w = P->rw;
  const int64_t n = P->L.ndof;
  if (w.VC && w.k == k && w.m == m && w.ndof == n) {
    if (w.p < p) TRY(recycle_width(P, st, p));
    if (p >= 2) {
      if (ensure_block_ws(w.bb, n, p, m / p + 1) != MXW_OK) {
        set_error("recycling workspace allocation failed");
        return MXW_ENOMEM;
      }
    }
    return MXW_OK;
  }
  w.mem.reset();
  w.bb.mem.reset();
  w.bb.H1 = nullptr;
  w.VC = w.W = w.R = w.YS = w.B1 = w.B2 = w.Tb = nullptr;
  w.npb = w.bnb = nullptr;
  w.xbuf = nullptr;
  w.dim = 0;
  w.k = k;
  w.m = m;
  w.ndof = n;
  const int maxv = m + 1, nblk = red_blocks(n);
  w.Zs = w.mem.alloc<double2>((size_t)m * n);
  w.U = w.mem.alloc<double2>((size_t)k * n);
  w.Ub = w.mem.alloc<double2>((size_t)k * n);
  w.Ut = w.mem.alloc<double2>((size_t)k * n);
  w.Ubt = w.mem.alloc<double2>((size_t)k * n);
  w.Ct = w.mem.alloc<double2>((size_t)k * n);
  w.h1 = w.mem.alloc<double2>(maxv);
  w.h2 = w.mem.alloc<double2>(maxv);
  w.part = w.mem.alloc<double2>((size_t)nblk * maxv);
  w.H = w.mem.alloc<double2>((size_t)maxv * m);
  w.sn = w.mem.alloc<double2>(maxv);
  w.g = w.mem.alloc<double2>(maxv + 1);
  w.y = w.mem.alloc<double2>(maxv);
  w.t = w.mem.alloc<double2>(kRecycleLd);
  w.G = w.mem.alloc<double2>((size_t)kRecycleLd * kRecycleMaxCycle);
  w.WVg = w.mem.alloc<double2>((size_t)kRecycleLd * k);
  w.UU = w.mem.alloc<double2>((size_t)k * k);
  w.Mc = w.mem.alloc<double2>((size_t)kRecycleLd * k);
  w.Mu = w.mem.alloc<double2>((size_t)kRecycleLd * k);
  w.mu = w.mem.alloc<double2>(kRecycleLd);
  w.cs = w.mem.alloc<double>(maxv);
  w.w0 = w.mem.alloc<double>(1);
  w.hn = w.mem.alloc<double>(1);
  w.npart = w.mem.alloc<double>(nblk);
  w.est = w.mem.alloc<double>(1);
  w.beta = w.mem.alloc<double>(1);
  w.jd = w.mem.alloc<int>(1);
  w.kd = w.mem.alloc<int>(1);
  w.info = w.mem.alloc<int>(1);
  bool ok = w.Zs && w.U && w.Ub && w.Ut && w.Ubt && w.Ct && w.h1 && w.h2 && w.part && w.H && w.sn && w.g && w.y &&
            w.t && w.G && w.WVg && w.UU && w.Mc && w.Mu && w.mu && w.cs && w.w0 && w.hn && w.npart && w.est && w.beta &&
            w.jd && w.kd && w.info;
  if (ok && !w.host) ok = hipHostMalloc((void**)&w.host, sizeof(double) * (8 + 2 * kRecycleMaxBlockP)) == hipSuccess;
  // Gram products of the deflation span up to m + p vectors against k
  if (ok) ok = ensure_block_ws(w.bw, n, k, (m + k) / k + 1) == MXW_OK;
  if (ok) ok = recycle_width(P, st, p) == MXW_OK;
  // block least squares: at most m / p block steps of p columns
  if (ok && p >= 2) ok = ensure_block_ws(w.bb, n, p, m / p + 1) == MXW_OK;
  if (!ok) {
    w.mem.reset();
    w.VC = nullptr;
    set_error("recycling workspace allocation failed");
    return MXW_ENOMEM;
  }
  return MXW_OK;
}

// host copy of a few device doubles (one synchronisation)
mxw_status fetch(hipStream_t st, double* host, std::initializer_list<const double*> src) {
  int i = 0;
  for (const double* p : src) HIP_CHECK(hipMemcpyAsync(host + i++, p, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  return MXW_OK;
}

mxw_status set_int(hipStream_t st, int* dev, int v) {
  HIP_CHECK(hipMemcpyAsync(dev, &v, sizeof(int), hipMemcpyHostToDevice, st));
  HIP_CHECK(hipStreamSynchronize(st));   // v lives on the host stack
  return MXW_OK;
}

// Carry the recycled space to a new operator: Ubar = M^{-1} U, C = A Ubar,
// C = Q R (Cholesky QR twice), C <- Q, U <- U R^{-1}, Ubar <- Ubar R^{-1}.
mxw_status recycle_refresh(mxw_problem* P, hipStream_t st) {
  RecycleWork& w = P->rw;
  const int64_t n = P->L.ndof;
  const int d = w.dim;
  apply_prec_dev(P, st, w.U, n, w.Ub, n, d, nullptr, w.YS, d >= 2 ? w.xbuf : nullptr);
  {
    ScopedKernelTimer tm("spmv");
    launch_spmv(st, P->spmv_group, n, P->rowptr, P->cols, P->vals, w.Ub, n, w.VC, n, nullptr, 0, d, nullptr);
  }
  TRY(cholqr2(P, w.bw, st, w.VC, w.Ct, w.VC, d));
  TRY(tall_gemm(P, st, w.U, d, w.bw.R1i, d, d, 1.0, 0.0, w.Ut));
  TRY(tall_gemm(P, st, w.Ut, d, w.bw.R2i, d, d, 1.0, 0.0, w.U));
  TRY(tall_gemm(P, st, w.Ub, d, w.bw.R1i, d, d, 1.0, 0.0, w.Ubt));
  TRY(tall_gemm(P, st, w.Ubt, d, w.bw.R2i, d, d, 1.0, 0.0, w.Ub));
  HIP_CHECK(hipGetLastError());
  w.gen = P->op_gen;
  ++w.refreshes;
  return MXW_OK;
}

// Deflated restart after a cycle with kk recycled vectors and jd Arnoldi
// steps: the new space from the harmonic Ritz vectors of the cycle.
// jd: Krylov vectors of the cycle (block steps x p); extra: rows of Gbar
// below kk + jd (1, or 0 after a breakdown, for one right-hand side; p for a
// block); nw: basis vectors [C, V] projected on U for W^H Vhat.
mxw_status recycle_deflate(mxw_problem* P, hipStream_t st, int kk, int jd, int extra, int nw) {
  RecycleWork& w = P->rw;
  const int64_t n = P->L.ndof;
  const int s = kk + jd, knew = std::min(w.k, s);
  if (knew == 0) return MXW_OK;
  if (kk) {
    TRY(gram(w.bw, n, st, w.VC, nw, w.U, kk, w.WVg));
    TRY(gram(w.bw, n, st, w.U, kk, w.U, kk, w.UU));
  }
  launch_rc_ritz(st, kk, jd, knew, extra, nw, w.G, w.WVg, w.UU, w.Mc, w.Mu, w.mu, w.info);
  HIP_CHECK(hipGetLastError());
  int info = 0;
  HIP_CHECK(hipMemcpyAsync(&info, w.info, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  if (info) {   // no usable Schur form: continue without a recycled space
    w.dim = 0;
    ++w.failures;
    return MXW_OK;
  }
  const int rows = s + extra;
  const int ld = kRecycleLd;
  TRY(tall_gemm(P, st, w.VC, rows, w.Mc, ld, knew, 1.0, 0.0, w.Ct));
  TRY(tall_gemm(P, st, w.U, kk, w.Mu, ld, knew, 1.0, 0.0, w.Ut));
  TRY(tall_gemm(P, st, w.VC + (int64_t)kk * n, jd, w.Mu + kk, ld, knew, 1.0, kk ? 1.0 : 0.0, w.Ut));
  TRY(tall_gemm(P, st, w.Ub, kk, w.Mu, ld, knew, 1.0, 0.0, w.Ubt));
  TRY(tall_gemm(P, st, w.Zs, jd, w.Mu + kk, ld, knew, 1.0, kk ? 1.0 : 0.0, w.Ubt));
  HIP_CHECK(hipMemcpyAsync(w.VC, w.Ct, sizeof(double2) * knew * n, hipMemcpyDeviceToDevice, st));
  HIP_CHECK(hipGetLastError());
  std::swap(w.U, w.Ut);
  std::swap(w.Ub, w.Ubt);
  w.dim = knew;
  w.gen = P->op_gen;
  ++w.deflations;
  return MXW_OK;
}

// One system A x = b by GCRO-DR with the problem's recycled space.
mxw_status recycle_solve_one(mxw_problem* P, hipStream_t st, const double2* b, double2* x, const mxw_solve_opts* opts,
                             int* iters_out, double* relres_out, bool* brk_any) {
  RecycleWork& w = P->rw;
  const int64_t n = P->L.ndof;
  const int m = w.m, maxv = m + 1;
  double* hb = w.host;
  HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double2) * n, st));
  launch_norm(st, n, b, n, w.npart, w.beta, 1, nullptr);
  TRY(fetch(st, hb, {w.beta}));
  const double bnorm = hb[0];
  w.history.clear();
  *iters_out = 0;
  *relres_out = 0.0;
  if (!(bnorm > 0)) return MXW_OK;
  if (w.dim && w.gen != P->op_gen) TRY(recycle_refresh(P, st));
  HIP_CHECK(hipMemcpyAsync(w.R, b, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
  int iters = 0;
  double relres = 1.0;
  bool conv = false;
  while (true) {
    const int kk = w.dim;
    if (kk) {   // minimal residual correction over range(U): t = C^H r
      TRY(set_int(st, w.kd, kk));
      launch_dots(st, n, kk, w.VC, 0, w.R, n, w.part, maxv, 1, nullptr);
      launch_reduce_dots(st, n, kk, w.part, w.t, maxv, 0, 1, nullptr);
      launch_xupdate(st, n, w.kd, w.Ub, 0, w.t, maxv, x, n, 1);
      launch_update(st, n, kk, w.VC, 0, w.R, n, w.t, maxv, 1, nullptr);
    }
    launch_norm(st, n, w.R, n, w.npart, w.beta, 1, nullptr);
    TRY(fetch(st, hb, {w.beta}));
    const double beta = hb[0];
    if (beta <= opts->tol * bnorm) {
      spmv_dev(P, st, x, w.W, b, 1, nullptr);
      launch_norm(st, n, w.W, n, w.npart, w.w0, 1, nullptr);
      TRY(fetch(st, hb, {w.w0}));
      relres = hb[0] / bnorm;
      if (relres <= opts->tol || beta == 0.0) {
        conv = relres <= opts->tol;
        break;
      }
    }
    const int steps = m - kk;
    launch_scale_inv(st, n, w.R, n, w.VC + (int64_t)kk * n, 0, w.beta, 1, nullptr);
    {
      std::vector<double2> g0(maxv + 1, make_double2(0.0, 0.0));
      g0[0] = make_double2(beta, 0.0);
      HIP_CHECK(hipMemcpyAsync(w.g, g0.data(), sizeof(double2) * g0.size(), hipMemcpyHostToDevice, st));
      HIP_CHECK(hipStreamSynchronize(st));
    }
    int jdone = 0;
    bool brk = false;
    for (int j = 0; j < steps; ++j) {
      double2* Vj = w.VC + (int64_t)(kk + j) * n;
      double2* Zj = w.Zs + (int64_t)j * n;
      const int nvec = kk + j + 1;
      apply_prec_dev(P, st, Vj, n, Zj, n, 1, nullptr, w.YS, nullptr);
      {
        ScopedKernelTimer tm("spmv");
        launch_spmv(st, P->spmv_group, n, P->rowptr, P->cols, P->vals, Zj, n, w.W, n, nullptr, 0, 1, nullptr);
      }
      launch_norm(st, n, w.W, n, w.npart, w.w0, 1, nullptr);
      // against [C, V_0..V_j] twice (CGS2); h1 = [B_j; h_j]
      launch_dots(st, n, nvec, w.VC, 0, w.W, n, w.part, maxv, 1, nullptr);
      launch_reduce_dots(st, n, nvec, w.part, w.h1, maxv, 0, 1, nullptr);
      launch_update(st, n, nvec, w.VC, 0, w.W, n, w.h1, maxv, 1, nullptr);
      launch_dots(st, n, nvec, w.VC, 0, w.W, n, w.part, maxv, 1, nullptr);
      launch_reduce_dots(st, n, nvec, w.part, w.h2, maxv, 0, 1, nullptr);
      launch_update(st, n, nvec, w.VC, 0, w.W, n, w.h2, maxv, 1, nullptr);
      launch_reduce_dots(st, n, nvec, w.part, w.h1, maxv, 1, 1, nullptr);
      launch_norm(st, n, w.W, n, w.npart, w.hn, 1, nullptr);
      launch_rc_save(st, kk, j, w.h1, w.hn, w.G);
      launch_givens(st, 1, j, maxv, w.h1 + kk, w.hn, w.H, m, w.cs, w.sn, w.g, w.est, nullptr);
      launch_scale_inv(st, n, w.W, n, w.VC + (int64_t)(nvec)*n, 0, w.hn, 1, nullptr);
      HIP_CHECK(hipGetLastError());
      TRY(fetch(st, hb, {w.est, w.hn, w.w0}));
      const double est = hb[0], hn = hb[1], w0 = hb[2];
      ++iters;
      jdone = j + 1;
      w.history.push_back(est / bnorm);
      brk = !(hn > 1e-14 * w0);
      if (brk) *brk_any = true;
      if (est <= opts->tol * bnorm || brk || iters >= opts->max_iters || !std::isfinite(est)) break;
    }
    // x += Z y - Ubar (B y)
    TRY(set_int(st, w.jd, jdone));
    launch_backsolve(st, 1, w.jd, maxv, w.H, m, w.g, w.y);
    launch_xupdate(st, n, w.jd, w.Zs, 0, w.y, maxv, x, n, 1);
    if (kk) {
      launch_rc_by(st, kk, w.jd, w.G, w.y, w.t);
      launch_xupdate(st, n, w.kd, w.Ub, 0, w.t, maxv, x, n, 1);
    }
    TRY(recycle_deflate(P, st, kk, jdone, brk ? 0 : 1, kk + jdone + 1));
    spmv_dev(P, st, x, w.R, b, 1, nullptr);
    launch_norm(st, n, w.R, n, w.npart, w.beta, 1, nullptr);
    HIP_CHECK(hipGetLastError());
    TRY(fetch(st, hb, {w.beta}));
    relres = hb[0] / bnorm;
    if (relres <= opts->tol) {
      conv = true;
      break;
    }
    if (iters >= opts->max_iters || !std::isfinite(relres)) break;
  }
  *iters_out = iters;
  *relres_out = relres;
  if (conv) return MXW_OK;
  return MXW_ENOTCONV;
}

// Block GCRO-DR: the p columns of B solved together with the problem's
// recycled space (Sec. 6: block and recycling strategies combined).  A cycle
// removes the block residual's part in range(C), runs block Arnoldi for
// (I - C C^H) A M^{-1} (block CGS2 against C and the previous blocks,
// Cholesky QR of each new block, the block Householder least squares of
// block GMRES), updates X += Z Y - Ubar (B Y) and replaces the space by the
// harmonic Ritz vectors of the cycle (Gbar with p rows below the Krylov
// part).  Iterations count block steps.
mxw_status recycle_solve_block(mxw_problem* P, hipStream_t st, int p, const double2* B, double2* X,
                               const mxw_solve_opts* opts, int32_t* iters_out, double* relres_out) {
  RecycleWork& w = P->rw;
  BlockWork& b = w.bb;
  const int64_t n = P->L.ndof;
  const int m = w.m, mb = b.m, ldE = (mb + 1) * p;
  double* hb = w.host;
  auto norms = [&](const double2* A, std::vector<double>& out) -> mxw_status {
    launch_norm(st, n, A, n, w.npb, w.bnb, p, nullptr);
    HIP_CHECK(hipMemcpyAsync(hb, w.bnb, sizeof(double) * p, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    out.assign(hb, hb + p);
    return MXW_OK;
  };
  std::vector<double> bn, rn(p, 1.0), est;
  TRY(norms(B, bn));
  for (int c = 0; c < p; ++c)
    if (!(bn[c] > 0)) {
      set_error("block recycling needs non-zero right-hand sides");
      return MXW_EINVAL;
    }
  w.history.clear();
  if (w.dim && w.gen != P->op_gen) TRY(recycle_refresh(P, st));
  HIP_CHECK(hipMemsetAsync(X, 0, sizeof(double2) * n * p, st));
  HIP_CHECK(hipMemcpyAsync(w.R, B, sizeof(double2) * n * p, hipMemcpyDeviceToDevice, st));
  auto below = [&](const std::vector<double>& v) {
    for (int c = 0; c < p; ++c)
      if (!(v[c] <= opts->tol * bn[c])) return false;
    return true;
  };
  int steps = 0;
  bool conv = false, bad = false;
  while (true) {
    const int kk = w.dim;
    if (kk) {   // minimal residual correction over range(U): T = C^H R
      TRY(gram(b, n, st, w.VC, kk, w.R, p, w.Tb));
      TRY(tall_gemm(P, st, w.Ub, kk, w.Tb, kk, p, 1.0, 1.0, X));
      TRY(tall_gemm(P, st, w.VC, kk, w.Tb, kk, p, -1.0, 1.0, w.R));
    }
    std::vector<double> pn;
    TRY(norms(w.R, pn));
    if (below(pn)) {   // verify with the true residual
      launch_spmv(st, P->spmv_group, n, P->rowptr, P->cols, P->vals, X, n, w.W, n, B, n, p, nullptr);
      TRY(norms(w.W, rn));
      if (below(rn)) {
        conv = true;
        break;
      }
    }
    const int nb = std::max(1, (m - kk) / p);
    double2* V = w.VC + (int64_t)kk * n;   // the cycle's blocks follow C
    TRY(cholqr2(P, b, st, w.R, w.W, V, p));
    launch_set_e(st, p, ldE, b.S, b.E);
    int jd = 0;
    for (int j = 0; j < nb; ++j) {
      double2* Vj = V + (int64_t)j * p * n;
      double2* Zj = w.Zs + (int64_t)j * p * n;
      const int Q = (j + 1) * p;
      apply_prec_dev(P, st, Vj, n, Zj, n, p, nullptr, w.YS, w.xbuf);
      {
        ScopedKernelTimer tm("spmv");
        launch_spmv(st, P->spmv_group, n, P->rowptr, P->cols, P->vals, Zj, n, w.W, n, nullptr, 0, p, nullptr);
      }
      for (int pass = 0; pass < 2; ++pass) {   // against C, then the previous blocks; twice
        double2* Bp = pass ? w.B2 : w.B1;
        double2* Hp = pass ? b.H2 : b.H1;
        if (kk) {
          TRY(gram(b, n, st, w.VC, kk, w.W, p, Bp));
          TRY(tall_gemm(P, st, w.VC, kk, Bp, kk, p, -1.0, 1.0, w.W));
        }
        TRY(gram(b, n, st, V, Q, w.W, p, Hp));
        TRY(tall_gemm(P, st, V, Q, Hp, Q, p, -1.0, 1.0, w.W));
      }
      TRY(cholqr2(P, b, st, w.W, w.R, V + (int64_t)Q * n, p));
      launch_rc_save_block(st, kk, j, p, w.B1, w.B2, b.H1, b.H2, b.S, w.G);
      launch_bls_step(st, j, p, mb, b.H1, b.H2, b.S, b.Hc, b.T, b.Rls, b.E, b.est);
      HIP_CHECK(hipGetLastError());
      HIP_CHECK(hipMemcpyAsync(hb, b.est, sizeof(double) * p, hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
      est.assign(hb, hb + p);
      ++steps;
      jd = j + 1;
      double worst = 0.0;
      for (int c = 0; c < p; ++c) {
        worst = std::max(worst, est[c] / bn[c]);
        if (!std::isfinite(est[c])) bad = true;
      }
      w.history.push_back(worst);
      if (below(est) || bad || steps >= opts->max_iters) break;
    }
    if (bad) {   // report the true residual of the iterate reached so far
      launch_spmv(st, P->spmv_group, n, P->rowptr, P->cols, P->vals, X, n, w.R, n, B, n, p, nullptr);
      HIP_CHECK(hipGetLastError());
      TRY(norms(w.R, rn));
      break;
    }
    // X += Z Y - Ubar (B Y)
    const int q = jd * p;
    launch_bls_solve(st, q, p, mb, b.Rls, b.E, b.Y);
    TRY(tall_gemm(P, st, w.Zs, q, b.Y, mb * p, p, 1.0, 1.0, X));
    if (kk) {
      launch_rc_by_block(st, kk, q, p, w.G, b.Y, mb * p, w.Tb);
      TRY(tall_gemm(P, st, w.Ub, kk, w.Tb, kk, p, 1.0, 1.0, X));
    }
    TRY(recycle_deflate(P, st, kk, q, p, kk + q + p));
    launch_spmv(st, P->spmv_group, n, P->rowptr, P->cols, P->vals, X, n, w.R, n, B, n, p, nullptr);
    HIP_CHECK(hipGetLastError());
    TRY(norms(w.R, rn));
    if (below(rn)) {
      conv = true;
      break;
    }
    bool finite = true;
    for (double v : rn) finite = finite && std::isfinite(v);
    if (steps >= opts->max_iters || !finite) {
      bad = bad || !finite;
      break;
    }
  }
  for (int c = 0; c < p; ++c) {
    if (iters_out) iters_out[c] = steps;
    if (relres_out) relres_out[c] = rn[c] / bn[c];
  }
  if (conv) return MXW_OK;
  if (bad) {
    set_error("block recycling: non-finite values before the tolerance");
    return MXW_EBREAKDOWN;
  }
  set_error("max_iters reached before the tolerance");
  return MXW_ENOTCONV;
}

}  // namespace

extern "C" {

mxw_status mxw_problem_create(mxw_ctx* ctx, const mxw_problem_desc* desc, void* stream, int32_t defer_factor,
                              mxw_problem** out) {
  if (!out) {
    set_error("out is NULL");
    return MXW_EINVAL;
  }
  *out = nullptr;
  std::shared_ptr<LayoutShared> S;
  try {
    S = std::make_shared<LayoutShared>();
    TRY(build_layout(desc, S->L));
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return MXW_ENOMEM;
  }
  return create_problem(ctx_of(ctx), S, nullptr, S->L.k0, desc->precision, desc->prec_variant, (hipStream_t)stream,
                        defer_factor, out);
}

mxw_status mxw_problem_create_from_layout(mxw_ctx* ctx, const mxw_layout* layout, const double* eps, double k0,
                                          int32_t precision, int32_t prec_variant, void* stream,
                                          int32_t defer_factor, mxw_problem** out) {
  if (!out || !layout) {
    set_error("NULL argument");
    return MXW_EINVAL;
  }
  *out = nullptr;
  return create_problem(ctx_of(ctx), layout->S, eps, k0 < 0 ? layout->S->L.k0 : k0, precision, prec_variant,
                        (hipStream_t)stream, defer_factor, out);
}

mxw_status mxw_problem_set_medium(mxw_problem* prob, const double* eps, double k0, void* stream) {
  TRY(check_problem(prob));
  const Layout& L = prob->L;
  if (!eps) eps = L.eps.data();
  if (k0 < 0) k0 = prob->k0;
  if (!std::isfinite(k0)) {
    set_error("k0 must be finite and >= 0");
    return MXW_EINVAL;
  }
  for (int64_t q = 0; q < 2 * L.nt; ++q)
    if (!std::isfinite(eps[q])) {
      set_error("non-finite permittivity");
      return MXW_EINVAL;
    }
  std::lock_guard<std::mutex> hold(prob->run);   // not while a solve uses the operator
  return assemble_medium(prob, eps, k0, (hipStream_t)stream, 0);
}

void mxw_problem_destroy(mxw_problem* prob) {
  if (!prob) return;
  { std::lock_guard<std::mutex> lk(prob->run); }   // an asynchronous solve still running ends first
  int cur = -1;
  const int dev = prob->device;
  const bool switched = hipGetDevice(&cur) == hipSuccess && cur != dev && hipSetDevice(dev) == hipSuccess;
  release_timing_events();   // waits only on recorded timing events, if any
  if (prob->kw.host) hipHostFree(prob->kw.host);
  delete prob;
  if (switched) hipSetDevice(cur);
}

mxw_status mxw_problem_get_info(const mxw_problem* prob, mxw_layout_info* info) {
  TRY(check_problem(prob));
  if (!info) {
    set_error("info is NULL");
    return MXW_EINVAL;
  }
  fill_info(prob->L, info);
  return MXW_OK;
}

mxw_status mxw_problem_factor(mxw_problem* prob, void* stream) {
  TRY(check_problem(prob));
  return factor_impl(prob, (hipStream_t)stream);
}

mxw_status mxw_problem_export_matrix(const mxw_problem* prob, double* vals) {
  TRY(check_problem(prob));
  if (!vals) {
    set_error("vals is NULL");
    return MXW_EINVAL;
  }
  HIP_CHECK(hipDeviceSynchronize());
  HIP_CHECK(hipMemcpy(vals, prob->vals, prob->L.cols.size() * 16, hipMemcpyDeviceToHost));
  return MXW_OK;
}

mxw_status mxw_problem_export_local(const mxw_problem* prob, int32_t s, double* a_s) {
  TRY(check_problem(prob));
  if (!a_s || s < 0 || s >= prob->L.n_sub) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  if (prob->factored) {
    set_error("local matrices are overwritten by their factors");
    return MXW_EINVAL;
  }
  const int64_t n = prob->L.sub_dof_ptr[s + 1] - prob->L.sub_dof_ptr[s];
  const int64_t ld = prob->S->h_lds[s];
  const size_t rsz = prob->mixed ? 4 : 8;
  std::vector<unsigned char> buf(2 * ld * n * rsz);
  HIP_CHECK(hipDeviceSynchronize());
  HIP_CHECK(hipMemcpy(buf.data(), (unsigned char*)prob->F + prob->S->h_foff[s] * rsz, buf.size(), hipMemcpyDeviceToHost));
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) {
      double re, im;
      if (prob->mixed) {
        re = ((float*)buf.data())[j * ld + i];
        im = ((float*)buf.data())[ld * n + j * ld + i];
      } else {
        re = ((double*)buf.data())[j * ld + i];
        im = ((double*)buf.data())[ld * n + j * ld + i];
      }
      a_s[2 * (j * n + i)] = re;
      a_s[2 * (j * n + i) + 1] = im;
    }
  return MXW_OK;
}

}  // extern "C"

namespace {

// Right-hand sides of mxw_problem_rhs.  given_work: a device buffer of at
// least n_imp_faces * nfloc complex128 for the face integrals of plane-wave
// and port sources (nullptr: allocated here when a source needs it).
mxw_status rhs_impl(mxw_problem* prob, int32_t nrhs, const mxw_source* src, double* b_dev, void* stream,
                    double2* given_work) {
  TRY(check_problem(prob));
  if (nrhs < 0 || (nrhs > 0 && (!src || !b_dev))) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const Layout& L = prob->L;
  const int64_t n = L.ndof;
  double2* b = (double2*)b_dev;
  HIP_CHECK(hipMemsetAsync(b, 0, sizeof(double2) * n * nrhs, st));
  double2* work = given_work;
  DevMem tmp(prob->ctx, st);   // the face integrals, if a source needs them and none were given
  auto face_work = [&]() -> mxw_status {
    if (work) return MXW_OK;
    work = tmp.alloc<double2>(L.imp_ft.size() * (size_t)L.basis.nfloc);
    if (!work) {
      set_error(tmp.why);
      return MXW_ENOMEM;
    }
    return MXW_OK;
  };
  for (int c = 0; c < nrhs; ++c) {
    const mxw_source& S = src[c];
    if (S.kind == MXW_SRC_DIPOLE) {
      // lowest-index element whose barycentric coordinates are all >= -1e-12
      int64_t found = -1;
      double lam[4] = {0, 0, 0, 0};
      for (int64_t t = 0; t < L.nt && found < 0; ++t) {
        const double* X[4];
        for (int q = 0; q < 4; ++q) X[q] = &L.xyz[3 * (int64_t)L.tets[4 * t + q]];
        double J[3][3];
        for (int r = 0; r < 3; ++r)
          for (int cc = 0; cc < 3; ++cc) J[r][cc] = X[cc + 1][r] - X[0][r];
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        const double y[3] = {S.pos[0] - X[0][0], S.pos[1] - X[0][1], S.pos[2] - X[0][2]};
        // Cramer's rule for J xi = y
        double xi[3];
        for (int k = 0; k < 3; ++k) {
          double M[3][3];
          for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc) M[r][cc] = (cc == k) ? y[r] : J[r][cc];
          xi[k] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                   M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
        }
        const double l0 = 1.0 - xi[0] - xi[1] - xi[2];
        if (l0 >= -1e-12 && xi[0] >= -1e-12 && xi[1] >= -1e-12 && xi[2] >= -1e-12) {
          found = t;
          lam[0] = l0;
          lam[1] = xi[0];
          lam[2] = xi[1];
          lam[3] = xi[2];
        }
      }
      if (found < 0) {
        set_error("dipole position outside the mesh");
        return MXW_EINVAL;
      }
      launch_rhs_dipole(st, prob->xyz, prob->tets, prob->tet_dofs, prob->phi, L.basis.nloc, found, lam, S.pol_re,
                        S.pol_im, b + (int64_t)c * n);
    } else if (S.kind == MXW_SRC_PLANEWAVE) {
      TRY(face_work());
      PlaneWaveArgs pa{(int)L.imp_ft.size(), n, prob->xyz, prob->ft_vert, prob->imp_ft, prob->imp_opp, prob->imp_beta,
                       prob->imp_eps, prob->fphi, L.basis.nfloc, prob->k0, prob->nq, prob->gx, prob->gw, prob->dof_ent,
                       prob->ent_imp_ptr, prob->ent_imps, prob->ft_dofs};
      launch_rhs_planewave(st, pa, S.pol_re, S.pol_im, S.dir, work, b + (int64_t)c * n);
    } else if (S.kind == MXW_SRC_PORT) {
      PortFrame pf;
      TRY(port_frame(S, pf));
      TRY(face_work());
      PlaneWaveArgs pa{(int)L.imp_ft.size(), n, prob->xyz, prob->ft_vert, prob->imp_ft, prob->imp_opp, prob->imp_beta,
                       prob->imp_eps, prob->fphi, L.basis.nfloc, prob->k0, prob->nq, prob->gx, prob->gw, prob->dof_ent,
                       prob->ent_imp_ptr, prob->ent_imps, prob->ft_dofs};
      launch_rhs_port(st, pa, pf.c, pf.u, pf.v, pf.a, pf.b, 0, work, nullptr, nullptr, b + (int64_t)c * n);
    } else {
      set_error("unknown source kind");
      return MXW_EINVAL;
    }
  }
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(st));   // before tmp goes back to the allocator
  return MXW_OK;
}

}  // namespace

// The no-allocation variant's face-integral buffer: one copy per device,
// held until the process ends.  Host code never passes `scratch` itself (on
// the host it is only a stand-in for the symbol): it looks up the device
// address once per device with hipGetSymbolAddress and uses that.
constexpr size_t kRhsScratchElems = (size_t)1 << 18;   // 4 MiB of complex128
static __device__ __align__(256) double2 scratch[kRhsScratchElems];

namespace {

static std::mutex g_scratch_mu;
static std::map<int, double2*> g_scratch_ptr;

mxw_status rhs_scratch(double2** out) {
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    double2* p = nullptr;
    HIP_CHECK(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("no device address for the right-hand-side scratch buffer");
      return MXW_EDEVICE;
    }
    it = g_scratch_ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return MXW_OK;
}

}  // namespace

extern "C" {

mxw_status mxw_problem_rhs(mxw_problem* prob, int32_t nrhs, const mxw_source* src, double* b_dev, void* stream) {
  return rhs_impl(prob, nrhs, src, b_dev, stream, nullptr);
}

mxw_status mxw_problem_rhs_noalloc(mxw_problem* prob, int32_t nrhs, const mxw_source* src, double* b_dev,
                                   void* stream) {
  TRY(check_problem(prob));
  const size_t need = prob->L.imp_ft.size() * (size_t)prob->L.basis.nfloc;
  if (need > kRhsScratchElems) {
    std::ostringstream os;
    os << "mxw_problem_rhs_noalloc: the face integrals need " << need * sizeof(double2)
       << " bytes, more than the fixed " << kRhsScratchElems * sizeof(double2) << "-byte buffer";
    set_error(os.str());
    return MXW_EINVAL;
  }
  if (prob->device >= 0) {
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    if (dev != prob->device) {
      set_error("mxw_problem_rhs_noalloc: the problem lives on another device than the current one");
      return MXW_EINVAL;
    }
  }
  double2* work = nullptr;
  TRY(rhs_scratch(&work));
  return rhs_impl(prob, nrhs, src, b_dev, stream, work);
}

mxw_status mxw_problem_apply_A(mxw_problem* prob, int32_t nrhs, const double* x_dev, double* y_dev, void* stream) {
  TRY(check_problem(prob));
  if (nrhs < 0 || (nrhs > 0 && (!x_dev || !y_dev))) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  if (nrhs >= kIlMinCols && nrhs <= interleaved_cols()) {
    // a block of columns as in the block solver: the matrix read once for
    // all of them, through a temporary interleaved copy
    DevMem tmp(prob->ctx, st);
    double2* xi = tmp.alloc<double2>((size_t)prob->L.ndof * interleaved_cols());
    if (!xi) {
      set_error(tmp.why);
      return MXW_ENOMEM;
    }
    ScopedKernelTimer tm("spmv");
    launch_spmm_interleaved(st, prob->L.ndof, nrhs, prob->rowptr, prob->cols, prob->vals, (const double2*)x_dev,
                            prob->L.ndof, xi, (double2*)y_dev, prob->L.ndof, nullptr, 0);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));   // before tmp goes back to the allocator
    return MXW_OK;
  }
  spmv_dev(prob, st, (const double2*)x_dev, (double2*)y_dev, nullptr, nrhs, nullptr);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(st));
  return MXW_OK;
}

mxw_status mxw_problem_apply_prec(mxw_problem* prob, int32_t nrhs, const double* v_dev, double* z_dev, void* stream) {
  TRY(check_problem(prob));
  if (nrhs < 0 || (nrhs > 0 && (!v_dev || !z_dev))) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  if (!prob->factored) {
    set_error("problem is not factorised");
    return MXW_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  DevMem tmp(prob->ctx, st);
  double2* ys = nullptr;
  void* xbuf = nullptr;
  if (gathered(prob->variant) && !(ys = tmp.alloc<double2>(prob->L.sum_ns * (size_t)std::max(1, nrhs)))) {
    set_error(tmp.why);
    return MXW_ENOMEM;
  }
  double2* vil = nullptr;
  if (!gathered(prob->variant) && nrhs >= 2) {
    const int nchunk = (nrhs + multi_chunk_cols() - 1) / multi_chunk_cols();
    xbuf = tmp.alloc<unsigned char>((size_t)nchunk * 2 * prob->L.sum_ns * multi_chunk_cols() * (prob->mixed ? 4 : 8));
    if (!xbuf) {
      set_error(tmp.why);
      return MXW_ENOMEM;
    }
    // a block of kIlMinCols..32 columns is gathered from an interleaved copy,
    // as in the block solver
    if (nrhs >= kIlMinCols && nrhs <= interleaved_cols()) {
      if (!(vil = tmp.alloc<double2>((size_t)prob->L.ndof * interleaved_cols()))) {
        set_error(tmp.why);
        return MXW_ENOMEM;
      }
      launch_to_interleaved(st, prob->L.ndof, nrhs, (const double2*)v_dev, prob->L.ndof, vil);
    }
  }
  apply_prec_dev(prob, st, (const double2*)v_dev, prob->L.ndof, (double2*)z_dev, prob->L.ndof, nrhs, nullptr, ys, xbuf,
                 vil);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(st));   // before tmp goes back to the allocator
  return MXW_OK;
}

mxw_status mxw_solve_rhs(mxw_problem* P, int32_t nrhs, const double* b_dev, const mxw_solve_opts* opts, void* stream,
                         double* x_dev, int32_t* iters_out, double* relres_out) {
  TRY(check_problem(P));
  if (nrhs < 1 || !b_dev || !x_dev || !opts) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  if (opts->restart < 1 || opts->restart > 200 || opts->max_iters < 1 || !(opts->tol > 0)) {
    set_error("invalid solve options (restart 1..200, max_iters >= 1, tol > 0)");
    return MXW_EINVAL;
  }
  if (opts->krylov != MXW_KRYLOV_PSEUDOBLOCK && opts->krylov != MXW_KRYLOV_BLOCK) {
    set_error("unknown Krylov mode");
    return MXW_EINVAL;
  }
  if (!P->factored) {
    set_error("problem is not factorised");
    return MXW_EINVAL;
  }
  std::lock_guard<std::mutex> hold(P->run);   // the Krylov workspace is the problem's
  if (opts->krylov == MXW_KRYLOV_BLOCK) {
    if (nrhs > max_block_p()) {
      set_error("block GMRES takes at most 32 right-hand sides per block");
      return MXW_EINVAL;
    }
    return block_solve(P, nrhs, (const double2*)b_dev, opts, (hipStream_t)stream, (double2*)x_dev, iters_out,
                       relres_out);
  }
  hipStream_t st = (hipStream_t)stream;
  const int m = opts->restart, maxv = m + 1;
  const int64_t n = P->L.ndof;
  TRY(ensure_krylov(P, nrhs, m));
  KrylovWork& k = P->kw;
  const double2* B = (const double2*)b_dev;
  double2* X = (double2*)x_dev;
  const int64_t vcol = (int64_t)maxv * n, zcol = (int64_t)m * n;
  double* hbuf = k.host;

  std::vector<double> bnorm(nrhs), beta(nrhs), relres(nrhs, 1.0);
  k.history.assign(nrhs, std::vector<double>());
  std::vector<int> iters(nrhs, 0), conv(nrhs, 0), act(nrhs, 0), jd(nrhs, 0);
  launch_norm(st, n, B, n, k.npart, k.beta, nrhs, nullptr);
  HIP_CHECK(hipMemcpyAsync(hbuf, k.beta, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  for (int c = 0; c < nrhs; ++c) {
    bnorm[c] = hbuf[c];
    beta[c] = bnorm[c];
    if (!(bnorm[c] > 0)) {
      conv[c] = 1;
      relres[c] = 0.0;
    }
  }
  HIP_CHECK(hipMemsetAsync(X, 0, sizeof(double2) * n * nrhs, st));
  HIP_CHECK(hipMemcpyAsync(k.Rv, B, sizeof(double2) * n * nrhs, hipMemcpyDeviceToDevice, st));
  mxw_status result = MXW_OK;
  bool breakdown_any = false;
  while (true) {
    int nact = 0;
    for (int c = 0; c < nrhs; ++c) {
      act[c] = (!conv[c] && iters[c] < opts->max_iters) ? 1 : 0;
      nact += act[c];
      jd[c] = 0;
    }
    if (nact == 0) break;
    HIP_CHECK(hipMemcpyAsync(k.active, act.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
    // V_0 = r / beta ; g = beta e_1
    launch_scale_inv(st, n, k.Rv, n, k.V, vcol, k.beta, nrhs, k.active);
    HIP_CHECK(hipMemsetAsync(k.g, 0, sizeof(double2) * nrhs * (maxv + 1), st));
    {
      std::vector<double2> g0((size_t)nrhs * (maxv + 1), make_double2(0.0, 0.0));
      for (int c = 0; c < nrhs; ++c) g0[(size_t)c * (maxv + 1)] = make_double2(beta[c], 0.0);
      HIP_CHECK(hipMemcpyAsync(k.g, g0.data(), sizeof(double2) * g0.size(), hipMemcpyHostToDevice, st));
      HIP_CHECK(hipStreamSynchronize(st));   // g0 lives on the host stack
    }
    for (int j = 0; j < m; ++j) {
      double2* Vj = k.V + (int64_t)j * n;
      double2* Zj = k.Z + (int64_t)j * n;
      // z_j = M^{-1} v_j (columns at stride vcol / zcol)
      // one Arnoldi step: z_j = M^{-1} v_j, w = A z_j, CGS2, ||w||, Givens, v_{j+1}
      auto step = [&](hipStream_t s) {
        apply_prec_dev(P, s, Vj, vcol, Zj, zcol, nrhs, k.active, k.YS, k.xbuf);
        {
          ScopedKernelTimer tm("spmv");
          launch_spmv(s, P->spmv_group, n, P->rowptr, P->cols, P->vals, Zj, zcol, k.W, n, nullptr, 0, nrhs,
                      k.active);
        }
        launch_norm(s, n, k.W, n, k.npart, k.w0, nrhs, k.active);
        launch_dots(s, n, j + 1, k.V, vcol, k.W, n, k.part, maxv, nrhs, k.active);
        launch_reduce_dots(s, n, j + 1, k.part, k.h1, maxv, 0, nrhs, k.active);
        launch_update(s, n, j + 1, k.V, vcol, k.W, n, k.h1, maxv, nrhs, k.active);
        launch_dots(s, n, j + 1, k.V, vcol, k.W, n, k.part, maxv, nrhs, k.active);
        launch_reduce_dots(s, n, j + 1, k.part, k.h2, maxv, 0, nrhs, k.active);
        launch_update(s, n, j + 1, k.V, vcol, k.W, n, k.h2, maxv, nrhs, k.active);
        launch_reduce_dots(s, n, j + 1, k.part, k.h1, maxv, 1, nrhs, k.active);   // h1 += h2
        launch_norm(s, n, k.W, n, k.npart, k.hn, nrhs, k.active);
        launch_givens(s, nrhs, j, maxv, k.h1, k.hn, k.H, m, k.cs, k.sn, k.g, k.est, k.active);
        launch_scale_inv(s, n, k.W, n, k.V + (int64_t)(j + 1) * n, vcol, k.hn, nrhs, k.active);
      };
      if (opts->use_graph) {
        // The step of index j is captured once per workspace and column count
        // and replayed: every argument is a fixed device address, a size or j;
        // the changing state (active columns, H, g) lives in device memory.
        // Capture runs on a private stream (the caller's may be the legacy
        // default stream, which cannot capture); replay runs on the caller's.
        if (k.graph_nrhs != nrhs) {
          k.drop_graphs();
          k.graph_nrhs = nrhs;
        }
        if ((int)k.graphs.size() < m) k.graphs.resize(m, nullptr);
        if (!k.graphs[j]) {
          if (!k.cap) HIP_CHECK(hipStreamCreateWithFlags(&k.cap, hipStreamNonBlocking));
          hipGraph_t g = nullptr;
          g_capturing = true;
          hipError_t ce = hipStreamBeginCapture(k.cap, hipStreamCaptureModeThreadLocal);
          if (ce == hipSuccess) {
            step(k.cap);
            ce = hipStreamEndCapture(k.cap, &g);
          }
          g_capturing = false;
          if (ce != hipSuccess) return dev_fail("graph capture", ce);
          const hipError_t ie = hipGraphInstantiate(&k.graphs[j], g, nullptr, nullptr, 0);
          hipGraphDestroy(g);
          if (ie != hipSuccess) {
            k.graphs[j] = nullptr;
            return dev_fail("hipGraphInstantiate", ie);
          }
        }
        HIP_CHECK(hipGraphLaunch(k.graphs[j], st));
      } else {
        step(st);
      }
      HIP_CHECK(hipGetLastError());
      HIP_CHECK(hipMemcpyAsync(hbuf, k.est, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipMemcpyAsync(hbuf + nrhs, k.hn, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipMemcpyAsync(hbuf + 2 * nrhs, k.w0, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
      int still = 0;
      bool changed = false;
      for (int c = 0; c < nrhs; ++c) {
        if (!act[c]) continue;
        iters[c]++;
        jd[c] = j + 1;
        const double est = hbuf[c], hn = hbuf[nrhs + c], w0 = hbuf[2 * nrhs + c];
        k.history[c].push_back(est / bnorm[c]);
        const bool brk = !(hn > 1e-14 * w0);
        if (brk) breakdown_any = true;
        if (est <= opts->tol * bnorm[c] || brk || iters[c] >= opts->max_iters || !std::isfinite(est)) {
          act[c] = 0;
          changed = true;
        } else {
          ++still;
        }
      }
      if (still == 0) break;
      if (changed) HIP_CHECK(hipMemcpyAsync(k.active, act.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
      if (changed) HIP_CHECK(hipStreamSynchronize(st));
    }
    // x += Z y; r = b - A x
    HIP_CHECK(hipMemcpyAsync(k.jd, jd.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
    launch_backsolve(st, nrhs, k.jd, maxv, k.H, m, k.g, k.y);
    launch_xupdate(st, n, k.jd, k.Z, zcol, k.y, maxv, X, n, nrhs);
    spmv_dev(P, st, X, k.Rv, B, nrhs, nullptr);
    launch_norm(st, n, k.Rv, n, k.npart, k.beta, nrhs, nullptr);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(hbuf, k.beta, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    for (int c = 0; c < nrhs; ++c) {
      if (conv[c]) continue;
      beta[c] = hbuf[c];
      relres[c] = beta[c] / bnorm[c];
      if (relres[c] <= opts->tol) conv[c] = 1;
    }
    bool any = false;
    for (int c = 0; c < nrhs; ++c)
      if (!conv[c] && iters[c] < opts->max_iters && std::isfinite(relres[c])) any = true;
    if (!any) break;
  }
  for (int c = 0; c < nrhs; ++c) {
    if (iters_out) iters_out[c] = iters[c];
    if (relres_out) relres_out[c] = relres[c];
    if (!conv[c]) result = breakdown_any ? MXW_EBREAKDOWN : MXW_ENOTCONV;
  }
  if (result == MXW_ENOTCONV) set_error("max_iters reached before the tolerance");
  if (result == MXW_EBREAKDOWN) set_error("Krylov breakdown before the tolerance");
  return result;
}

mxw_status mxw_solve(mxw_problem* P, int32_t nrhs, const mxw_source* src, const mxw_solve_opts* opts, void* stream,
                     double* E_out, int32_t E_out_is_device, int32_t* iters_out, double* relres_out) {
  TRY(check_problem(P));
  if (nrhs < 1 || !src || !opts || !E_out) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = P->L.ndof;
  DevMem tmp(P->ctx, st);
  double2* b = tmp.alloc<double2>((size_t)n * nrhs);
  double2* x = E_out_is_device ? (double2*)E_out : (b ? tmp.alloc<double2>((size_t)n * nrhs) : nullptr);
  if (!b || !x) {
    set_error(tmp.why);
    return MXW_ENOMEM;
  }
  mxw_status s = mxw_problem_rhs(P, nrhs, src, (double*)b, stream);
  if (s == MXW_OK || s == MXW_ENOTCONV) s = mxw_solve_rhs(P, nrhs, (double*)b, opts, stream, (double*)x, iters_out, relres_out);
  if (!E_out_is_device && (s == MXW_OK || s == MXW_ENOTCONV || s == MXW_EBREAKDOWN)) {
    hipMemcpyAsync(E_out, x, sizeof(double2) * n * nrhs, hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
  }
  hipStreamSynchronize(st);   // before tmp goes back to the allocator
  return s;
}

}  // extern "C"

struct mxw_ticket {
  std::thread th;
  std::atomic<int> done{0};
  mxw_status status = MXW_OK;
  std::string msg;
  std::vector<mxw_source> src;
  mxw_solve_opts opts{};
};

extern "C" {

mxw_status mxw_solve_async(mxw_problem* P, int32_t nrhs, const mxw_source* src, const mxw_solve_opts* opts,
                           void* stream, double* E_out, int32_t E_out_is_device, int32_t* iters_out,
                           double* relres_out, mxw_ticket** ticket) {
  TRY(check_problem(P));
  if (!ticket || nrhs < 1 || !src || !opts || !E_out) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  *ticket = nullptr;
  std::unique_ptr<mxw_ticket> T(new (std::nothrow) mxw_ticket());
  if (!T) {
    set_error("host allocation failed");
    return MXW_ENOMEM;
  }
  T->src.assign(src, src + nrhs);
  T->opts = *opts;
  mxw_ticket* t = T.get();
  const int dev = P->device;
  try {
    T->th = std::thread([=] {
      mxw_status st = (hipSetDevice(dev) == hipSuccess)
                          ? mxw_solve(P, nrhs, t->src.data(), &t->opts, stream, E_out, E_out_is_device, iters_out,
                                      relres_out)
                          : dev_fail("hipSetDevice", hipGetLastError());
      t->status = st;
      if (st != MXW_OK) t->msg = g_err;
      t->done.store(1, std::memory_order_release);
    });
  } catch (const std::system_error&) {
    set_error("could not start the solve thread");
    return MXW_ENOMEM;
  }
  *ticket = T.release();
  return MXW_OK;
}

mxw_status mxw_ticket_poll(mxw_ticket* t, int32_t* done) {
  if (!t || !done) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  *done = t->done.load(std::memory_order_acquire);
  return MXW_OK;
}

mxw_status mxw_ticket_wait(mxw_ticket* t) {
  if (!t) {
    set_error("ticket is NULL");
    return MXW_EINVAL;
  }
  if (t->th.joinable()) t->th.join();
  if (t->status != MXW_OK) set_error(t->msg);
  return t->status;
}

void mxw_ticket_destroy(mxw_ticket* t) {
  if (!t) return;
  if (t->th.joinable()) t->th.join();
  delete t;
}

mxw_status mxw_problem_forget_factors(mxw_problem* P) {
  TRY(check_problem(P));
  std::lock_guard<std::mutex> hold(P->run);
  P->hash_valid = false;
  return MXW_OK;
}

mxw_status mxw_problem_factor_stats(const mxw_problem* P, int32_t* refactored_last, int64_t* refactored_total,
                                    int64_t* kept_total) {
  TRY(check_problem(P));
  if (refactored_last) *refactored_last = (int32_t)P->refactor_last;
  if (refactored_total) *refactored_total = P->refactor_total;
  if (kept_total) *kept_total = P->kept_total;
  return MXW_OK;
}

mxw_status mxw_problem_device_bytes(const mxw_problem* P, uint64_t* bytes) {
  TRY(check_problem(P));
  if (!bytes) {
    set_error("bytes is NULL");
    return MXW_EINVAL;
  }
  *bytes = P->mem.bytes + P->kw.mem.bytes + P->bw.mem.bytes + P->rw.mem.bytes + P->rw.bw.mem.bytes +
           P->rw.bb.mem.bytes;
  return MXW_OK;
}

mxw_status mxw_problem_set_tiles(mxw_problem* P, int32_t spmv_group, int32_t multi_ku, int32_t lu_ku,
                                 int32_t multi_rows, int32_t lu_launch) {
  TRY(check_problem(P));
  const bool g_ok = spmv_group == 0 || spmv_group == 4 || spmv_group == 8 || spmv_group == 16 || spmv_group == 32;
  const bool k_ok = multi_ku == 0 || multi_ku == 4 || multi_ku == 8;
  const bool l_ok = lu_ku == 0 || lu_ku == 4 || lu_ku == 8;
  const bool r_ok = multi_rows == 0 || multi_rows == 64 || multi_rows == 128;
  const bool q_ok = lu_launch >= 0 && lu_launch <= 2;
  if (!g_ok || !k_ok || !l_ok || !r_ok || !q_ok) {
    set_error("spmv_group must be 0, 4, 8, 16 or 32, multi_ku and lu_ku 0, 4 or 8, multi_rows 0, 64 or 128, "
              "lu_launch 0, 1 or 2");
    return MXW_EINVAL;
  }
  if (lu_launch) P->lu_persistent = lu_launch == 2;
  if (spmv_group) P->spmv_group = spmv_group;
  if (multi_ku) P->multi_ku = multi_ku;
  if (lu_ku) P->lu_ku = lu_ku;
  if (multi_rows) P->multi_rows = multi_rows;
  if (P->multi_rows == 128) P->multi_ku = 8;   // 128-row passes take 8-wide slices
  P->kw.drop_graphs();   // captured steps hold the previous tile kernels
  P->bw.drop_graphs();
  return MXW_OK;
}

mxw_status mxw_problem_tune(mxw_problem* P, int32_t nrhs, void* stream, mxw_tuning* out) {
  TRY(check_problem(P));
  if (nrhs < 1 || nrhs > 4096) {
    set_error("nrhs must be in 1..4096");
    return MXW_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = P->L.ndof;
  DevMem tmp(P->ctx, st);
  double2* x = tmp.alloc<double2>((size_t)n * nrhs);
  double2* y = tmp.alloc<double2>((size_t)n * nrhs);
  if (!x || !y) {
    set_error("device allocation failed (tuning buffers)");
    return MXW_ENOMEM;
  }
  HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double2) * n * nrhs, st));
  struct Events {   // destroyed on every return path
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) hipEventDestroy(a);
      if (b) hipEventDestroy(b);
    }
  } ev;
  HIP_CHECK(hipEventCreate(&ev.a));
  HIP_CHECK(hipEventCreate(&ev.b));
  hipEvent_t ea = ev.a, eb = ev.b;
  // average of 3 launches after one untimed launch
  auto time_ms = [&](const std::function<void()>& fn) -> double {
    fn();
    hipEventRecord(ea, st);
    for (int r = 0; r < 3; ++r) fn();
    hipEventRecord(eb, st);
    hipEventSynchronize(eb);
    float ms = 0.f;
    hipEventElapsedTime(&ms, ea, eb);
    return ms / 3.0;
  };
  mxw_tuning t{};
  const int groups[4] = {4, 8, 16, 32};
  int best = 0;
  for (int g = 0; g < 4; ++g) {
    t.spmv_ms[g] = time_ms([&] {
      launch_spmv(st, groups[g], n, P->rowptr, P->cols, P->vals, x, n, y, n, nullptr, 0, nrhs, nullptr);
    });
    if (t.spmv_ms[g] < t.spmv_ms[best]) best = g;
  }
  P->spmv_group = groups[best];
  t.spmv_group = P->spmv_group;
  if (nrhs >= 2 && !gathered(P->variant) && P->factored) {
    const int nchunk = (nrhs + multi_chunk_cols() - 1) / multi_chunk_cols();
    void* xbuf = tmp.alloc<unsigned char>((size_t)nchunk * 2 * P->L.sum_ns * multi_chunk_cols() *
                                          (P->mixed ? 4 : 8));
    if (!xbuf) {
      set_error("device allocation failed (tuning scratch)");
      return MXW_ENOMEM;
    }
    const int kus[2] = {4, 8};
    P->multi_rows = 64;
    for (int q = 0; q < 2; ++q) {
      P->multi_ku = kus[q];
      t.multi_ms[q] = time_ms([&] { apply_prec_dev(P, st, x, n, y, n, nrhs, nullptr, nullptr, xbuf); });
    }
    P->multi_ku = t.multi_ms[0] < t.multi_ms[1] ? kus[0] : kus[1];
    if (P->mixed) {   // 128-row passes (8-wide slices; FP32 only: in FP64 the LDS leaves one workgroup per CU)
      P->multi_rows = 128;
      const int ku_keep = P->multi_ku;
      P->multi_ku = 8;
      t.multi_tall_ms = time_ms([&] { apply_prec_dev(P, st, x, n, y, n, nrhs, nullptr, nullptr, xbuf); });
      if (t.multi_tall_ms < std::min(t.multi_ms[0], t.multi_ms[1])) {
        P->multi_ku = 8;
      } else {
        P->multi_rows = 64;
        P->multi_ku = ku_keep;
      }
    }
  }
  t.multi_ku = P->multi_ku;
  t.multi_rows = P->multi_rows;
  if (P->mixed && P->factored) {
    // the LU is in place: each trial re-assembles the local matrices first
    const int kus[2] = {4, 8};
    for (int q = 0; q < 2; ++q) {
      P->lu_ku = kus[q];
      TRY(build_local_and_factor<float>(P, st, false));
      hipEventRecord(ea, st);
      launch_lu<float>(st, P->L.n_sub, (float*)P->F, P->foff, P->nsz, P->lds, P->perm, P->poff,
                       (float*)P->lu_scratch, P->info, P->order, P->lu_ku, lu_queue(P));
      hipEventRecord(eb, st);
      hipEventSynchronize(eb);
      float ms = 0.f;
      hipEventElapsedTime(&ms, ea, eb);
      t.lu_ms[q] = ms;
    }
    const int best = t.lu_ms[0] < t.lu_ms[1] ? kus[0] : kus[1];
    if (best != P->lu_ku) {
      P->lu_ku = best;
      P->factored = false;
      TRY(build_local_and_factor<float>(P, st, false));
      TRY(factor_impl(P, st));
    } else {
      ++P->op_gen;   // new factors (same operator up to rounding)
    }
  }
  t.lu_ku = P->mixed ? P->lu_ku : 4;
  if (P->factored) {
    // the LU's launch: one workgroup per subdomain or the persistent queue
    // (each trial re-assembles the local matrices first)
    const bool keep = P->lu_persistent;
    for (int q = 0; q < 2; ++q) {
      P->lu_persistent = q == 1;
      if (P->mixed)
        TRY(build_local_and_factor<float>(P, st, false));
      else
        TRY(build_local_and_factor<double>(P, st, false));
      hipEventRecord(ea, st);
      if (P->mixed)
        launch_lu<float>(st, P->L.n_sub, (float*)P->F, P->foff, P->nsz, P->lds, P->perm, P->poff,
                         (float*)P->lu_scratch, P->info, P->order, P->lu_ku, lu_queue(P));
      else
        launch_lu<double>(st, P->L.n_sub, (double*)P->F, P->foff, P->nsz, P->lds, P->perm, P->poff,
                          (double*)P->lu_scratch, P->info, P->order, P->lu_ku, lu_queue(P));
      hipEventRecord(eb, st);
      hipEventSynchronize(eb);
      float ms = 0.f;
      hipEventElapsedTime(&ms, ea, eb);
      t.lu_launch_ms[q] = ms;
    }
    P->lu_persistent = t.lu_launch_ms[1] <= t.lu_launch_ms[0];
    (void)keep;
    ++P->op_gen;   // new factors (the same bits: both launches run the same per-subdomain code)
  }
  t.lu_launch = P->lu_persistent ? 2 : 1;
  P->kw.drop_graphs();   // captured steps hold the previous tile kernels
  P->bw.drop_graphs();
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(st));
  if (out) *out = t;
  return MXW_OK;
}

mxw_status mxw_smatrix(mxw_problem* P, int32_t nports, const mxw_source* ports, int32_t nsol, const double* X_dev,
                       void* stream, double* S_dev) {
  TRY(check_problem(P));
  if (nports < 1 || nsol < 1 || !ports || !X_dev || !S_dev) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  std::vector<PortFrame> pf(nports);
  for (int i = 0; i < nports; ++i) TRY(port_frame(ports[i], pf[i]));
  hipStream_t st = (hipStream_t)stream;
  const Layout& L = P->L;
  const int64_t n = L.ndof;
  const int nimp = (int)L.imp_ft.size();
  constexpr int kChunk = 32;
  DevMem tmp(P->ctx, st);
  double2* W = tmp.alloc<double2>((size_t)kChunk * n);
  double2* work = tmp.alloc<double2>(std::max<size_t>(1, (size_t)nimp * L.basis.nfloc));
  double* fnorm = tmp.alloc<double>(std::max(1, nimp));
  double* den = tmp.alloc<double>(kChunk);
  double2* num = tmp.alloc<double2>((size_t)kChunk * nsol);
  BlockWork bw;
  bw.mem.ctx = P->ctx;
  if (!W || !work || !fnorm || !den || !num || ensure_block_ws(bw, n, kChunk, (nsol + kChunk - 1) / kChunk + 1) != MXW_OK) {
    set_error("device allocation failed (S-matrix buffers)");
    return MXW_ENOMEM;
  }
  PlaneWaveArgs pa{nimp, n, P->xyz, P->ft_vert, P->imp_ft, P->imp_opp, P->imp_beta, P->imp_eps, P->fphi, L.basis.nfloc,
                   P->k0, P->nq, P->gx, P->gw, P->dof_ent, P->ent_imp_ptr, P->ent_imps, P->ft_dofs};
  std::vector<double> dh(kChunk);
  for (int i0 = 0; i0 < nports; i0 += kChunk) {
    const int np = std::min(kChunk, nports - i0);
    HIP_CHECK(hipMemsetAsync(W, 0, sizeof(double2) * np * n, st));   // the face integrals are added into W
    for (int i = 0; i < np; ++i)
      launch_rhs_port(st, pa, pf[i0 + i].c, pf[i0 + i].u, pf[i0 + i].v, pf[i0 + i].a, pf[i0 + i].b, 1, work, fnorm,
                      den + i, W + (int64_t)i * n);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(dh.data(), den, sizeof(double) * np, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    for (int i = 0; i < np; ++i)
      if (!(dh[i] > 0)) {
        std::ostringstream os;
        os << "port " << i0 + i << " has no impedance face";
        set_error(os.str());
        return MXW_EINVAL;
      }
    // num[i nsol + j] = sum_k conj(X_j[k]) W_i[k]
    TRY(gram(bw, n, st, (const double2*)X_dev, nsol, W, np, num));
    launch_smatrix_finish(st, nsol, np, num, den, (double2*)S_dev + (int64_t)i0 * nsol);
    HIP_CHECK(hipGetLastError());
  }
  HIP_CHECK(hipStreamSynchronize(st));
  return MXW_OK;
}

mxw_status mxw_solve_recycle(mxw_problem* P, int32_t nrhs, const double* b_dev, const mxw_solve_opts* opts, int32_t k,
                             void* stream, double* x_dev, int32_t* iters_out, double* relres_out) {
  TRY(check_problem(P));
  if (nrhs < 1 || !b_dev || !x_dev || !opts) {
    set_error("invalid argument");
    return MXW_EINVAL;
  }
  if (k < 1 || k > kRecycleMaxK || opts->restart <= k || opts->restart > kRecycleMaxCycle || opts->max_iters < 1 ||
      !(opts->tol > 0)) {
    set_error("invalid recycling options (1 <= k <= 32, k < restart <= 64, max_iters >= 1, tol > 0)");
    return MXW_EINVAL;
  }
  if (!P->factored) {
    set_error("problem is not factorised");
    return MXW_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> hold(P->run);
  if (opts->krylov == MXW_KRYLOV_BLOCK && nrhs >= 2) {
    // a cycle holds C (k vectors) and at least one block step: k + nrhs <= restart
    if (nrhs > kRecycleMaxBlockP || opts->restart + nrhs > kRecycleLd || k + nrhs > opts->restart) {
      set_error("block recycling takes 2..16 right-hand sides, k + nrhs <= restart and restart + nrhs <= 65");
      return MXW_EINVAL;
    }
    TRY(ensure_recycle(P, st, k, opts->restart, nrhs));
    return recycle_solve_block(P, st, nrhs, (const double2*)b_dev, (double2*)x_dev, opts, iters_out, relres_out);
  }
  TRY(ensure_recycle(P, st, k, opts->restart));
  const int64_t n = P->L.ndof;
  mxw_status result = MXW_OK;
  bool brk = false;
  for (int c = 0; c < nrhs; ++c) {
    int it = 0;
    double rr = 0.0;
    const mxw_status r = recycle_solve_one(P, st, (const double2*)b_dev + (int64_t)c * n,
                                           (double2*)x_dev + (int64_t)c * n, opts, &it, &rr, &brk);
    if (iters_out) iters_out[c] = it;
    if (relres_out) relres_out[c] = rr;
    if (r == MXW_ENOTCONV) result = brk ? MXW_EBREAKDOWN : MXW_ENOTCONV;
    else if (r != MXW_OK) return r;
  }
  if (result == MXW_ENOTCONV) set_error("max_iters reached before the tolerance");
  if (result == MXW_EBREAKDOWN) set_error("Krylov breakdown before the tolerance");
  return result;
}

mxw_status mxw_recycle_reset(mxw_problem* P) {
  TRY(check_problem(P));
  P->rw.dim = 0;
  return MXW_OK;
}

mxw_status mxw_recycle_export(mxw_problem* P, int32_t* dim, double* U_dev, double* Ubar_dev, double* C_dev,
                              void* stream) {
  TRY(check_problem(P));
  const RecycleWork& w = P->rw;
  const int d = w.VC ? w.dim : 0;
  if (dim) *dim = d;
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = sizeof(double2) * (size_t)d * P->L.ndof;
  if (d && U_dev) HIP_CHECK(hipMemcpyAsync(U_dev, w.U, bytes, hipMemcpyDeviceToDevice, st));
  if (d && Ubar_dev) HIP_CHECK(hipMemcpyAsync(Ubar_dev, w.Ub, bytes, hipMemcpyDeviceToDevice, st));
  if (d && C_dev) HIP_CHECK(hipMemcpyAsync(C_dev, w.VC, bytes, hipMemcpyDeviceToDevice, st));
  HIP_CHECK(hipStreamSynchronize(st));
  return MXW_OK;
}

mxw_status mxw_recycle_stats(const mxw_problem* P, int64_t* refreshes, int64_t* deflations, int64_t* failures) {
  TRY(check_problem(P));
  if (refreshes) *refreshes = P->rw.refreshes;
  if (deflations) *deflations = P->rw.deflations;
  if (failures) *failures = P->rw.failures;
  return MXW_OK;
}

mxw_status mxw_solve_history(const mxw_problem* P, int32_t col, double* out, int32_t max_len, int32_t* len) {
  TRY(check_problem(P));
  if (!len || col < 0 || col >= (int32_t)P->kw.history.size()) {
    set_error("invalid argument (no solve recorded for this column)");
    return MXW_EINVAL;
  }
  const auto& h = P->kw.history[col];
  *len = (int32_t)h.size();
  if (out)
    for (int32_t q = 0; q < std::min<int32_t>(max_len, (int32_t)h.size()); ++q) out[q] = h[q];
  return MXW_OK;
}

mxw_status mxw_set_timing(int32_t enabled) {
  g_timing = enabled != 0;
  return MXW_OK;
}

mxw_status mxw_get_timing(const char* name, double* total_ms, int64_t* launches) {
  if (!name || !total_ms || !launches) {
    set_error("NULL argument");
    return MXW_EINVAL;
  }
  flush_timing();
  std::lock_guard<std::mutex> lk(g_tmu);
  auto it = g_totals.find(name);
  *total_ms = it == g_totals.end() ? 0.0 : it->second.first;
  *launches = it == g_totals.end() ? 0 : it->second.second;
  return MXW_OK;
}

mxw_status mxw_reset_timing(void) {
  flush_timing();
  std::lock_guard<std::mutex> lk(g_tmu);
  g_totals.clear();
  return MXW_OK;
}

}  // extern "C"
