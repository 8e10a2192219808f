// Host side of the ISDF library: context, memory planner, the fit / Coulomb
// kernel / fragment-ERI pipelines and the serving thread, behind the C ABI
// declared in include/isdf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/isdf.h"
#include "kernels.hpp"

namespace {

const char* kVersion = "isdf-gfx950 0.1";


struct Fail {
  isdf_status st;
  std::string msg;
};

#define HIPCHK(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw Fail{ISDF_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)};        \
  } while (0)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Workspace of isdf_fragment_eri_static: a file-scope device array that the
// library never allocates or frees (each GPU that loads the library holds
// its own copy for the life of the process).  Its first STATIC_DESC_BYTES
// hold the descriptors of a call, the rest the fragment workspace.  Host
// code never passes `scratch` itself to a kernel: it takes the device
// address of this GPU's copy from hipGetSymbolAddress once per device
// (scratch_ptr) and passes that.
constexpr size_t STATIC_SCRATCH_BYTES = ISDF_STATIC_SCRATCH_BYTES;
constexpr size_t STATIC_DESC_BYTES = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;    // device -> address of its copy of scratch

// Address of the current device's copy of scratch (looked up once per device).
void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    throw Fail{ISDF_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
  }
  g_scratch_ptr[device] = ptr;
  return ptr;
}

// Device allocation that is freed with its owner.
// A buffer attached to caller-provided memory (attach) never allocates or
// frees: asking it for more than it holds is ISDF_E_NOMEM.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool fixed = false;
  void attach(void* ptr, size_t b) {
    release();
    p = ptr;
    bytes = b;
    fixed = true;
  }
  void alloc(size_t b) {
    if (fixed)
      throw Fail{ISDF_E_NOMEM, "needs " + std::to_string(b) + " bytes of the " + std::to_string(bytes) +
                                   "-byte static workspace"};
    release();
    if (b == 0) return;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Fail{ISDF_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed"};
    }
    bytes = b;
  }
  void ensure(size_t b) {
    if (b > bytes) alloc(b);
  }
  void release() {
    if (p && !fixed) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    fixed = false;
  }
  ~DevBuf() { release(); }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    if (hipHostMalloc(&p, b, 0) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Fail{ISDF_E_NOMEM, "pinned host allocation failed"};
    }
    bytes = b;
  }
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
};

// Descriptor arena: GEMM descriptors and small tables are written to pinned
// host memory and copied to device memory on the launching stream.  Reset
// only after the stream has drained.
// The host copy is pinned, so a queued copy reads it when it executes: reset
// waits for the stream (the previous user of the arena may still have copies
// queued), and reserve sizes the arena for a whole pass before its first put
// (earlier device pointers must stay valid while the pass is enqueued).
struct Arena {
  PinnedBuf host;
  DevBuf dev;
  size_t used = 0;
  // attached to caller-provided device memory: descriptors are staged in
  // pageable host memory and nothing is allocated on the device
  std::vector<char> pageable;
  void attach(void* dev_ptr, size_t cap) {
    dev.attach(dev_ptr, cap);
    pageable.assign(cap, 0);
    used = 0;
  }
  char* host_ptr() { return dev.fixed ? pageable.data() : (char*)host.p; }
  size_t host_cap() const { return dev.fixed ? pageable.size() : host.bytes; }
  void reset(hipStream_t s) {
    HIPCHK(hipStreamSynchronize(s));
    used = 0;
  }
  // Capacity for `bytes` of puts (each put adds at most 255 bytes of
  // alignment); the stream has drained (reset) and nothing was put yet.
  void reserve(size_t bytes) {
    if (used != 0) throw Fail{ISDF_E_INVALID, "descriptor arena reserved after a put"};
    if (dev.fixed) {
      if (bytes > dev.bytes)
        throw Fail{ISDF_E_NOMEM, "descriptors need " + std::to_string(bytes) + " bytes of the " +
                                     std::to_string(dev.bytes) + "-byte static descriptor region"};
      return;
    }
    const size_t cap = std::max<size_t>(1 << 20, bytes);
    if (host.bytes < cap) host.ensure(cap);
    if (dev.bytes < cap) dev.ensure(cap);
  }
  template <class T> T* put(const T* src, size_t n, hipStream_t s) {
    size_t bytes = n * sizeof(T);
    size_t off = (used + 255) & ~size_t(255);
    if (off + bytes > host_cap() || off + bytes > dev.bytes) {
      if (used != 0 || dev.fixed) throw Fail{ISDF_E_NOMEM, "descriptor arena exhausted"};
      size_t cap = std::max<size_t>(1 << 20, 2 * bytes);
      host.ensure(cap);
      dev.ensure(cap);
      off = 0;
    }
    memcpy(host_ptr() + off, src, bytes);
    HIPCHK(hipMemcpyAsync((char*)dev.p + off, host_ptr() + off, bytes, hipMemcpyHostToDevice, s));
    used = off + bytes;
    return reinterpret_cast<T*>((char*)dev.p + off);
  }
};

int g_max_blocks = 0;
int max_gemm_blocks() {
  if (g_max_blocks == 0) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
      hipDeviceProp_t pr;
      if (hipGetDeviceProperties(&pr, dev) == hipSuccess) cus = pr.multiProcessorCount;
    }
    g_max_blocks = cus * 8;
  }
  return g_max_blocks;
}

// Workgroups per CU of the persistent GEMM launches issued by this thread (0:
// the default of max_gemm_blocks); the fragment pipeline sets it from its
// context's tuned value for the duration of a batch.
thread_local int t_wg_per_cu = 0;
int gemm_blocks() {
  if (t_wg_per_cu <= 0) return max_gemm_blocks();
  return max_gemm_blocks() / 8 * t_wg_per_cu;
}
struct WgScope {
  int old;
  explicit WgScope(int v) : old(t_wg_per_cu) { t_wg_per_cu = v; }
  ~WgScope() { t_wg_per_cu = old; }
};

void run_gemm(Arena& ar, int prec, int layout, std::vector<GemmDesc>& d, hipStream_t s) {
  long long total = gemm_plan(d.data(), (int)d.size());
  if (total == 0) return;
  GemmDesc* dd = ar.put(d.data(), d.size(), s);
  HIPCHK(gemm_launch(prec, layout, dd, (int)d.size(), total, gemm_blocks(), s));
}

// mark(true) / mark(false) bracket each kernel launch when given (kernel timing)
typedef std::function<void(bool)> LaunchMark;

void run_nt(Arena& ar, int prec, int conj, std::vector<NtDesc>& d, hipStream_t s, int kind = 0,
            const LaunchMark& mark = nullptr) {
  long long total = nt_plan(d.data(), (int)d.size());
  if (total == 0) return;
  NtDesc* dd = ar.put(d.data(), d.size(), s);
  if (mark) mark(true);
  HIPCHK(nt_launch(prec, conj, dd, (int)d.size(), total, gemm_blocks(), s, kind));
  if (mark) mark(false);
}

// Upload big-tile descriptors once and launch them for each K segment.
void run_big(Arena& ar, int prec, int conj, std::vector<NtDesc>& d, int nseg, hipStream_t s, int kind,
             const LaunchMark& mark = nullptr) {
  long long total = big_plan(d.data(), (int)d.size());
  if (total == 0) return;
  NtDesc* dd = ar.put(d.data(), d.size(), s);
  for (int seg = 0; seg < nseg; ++seg) {
    if (mark) mark(true);
    // the ring pipeline of the bf16 kernels (one workgroup a CU): for U^q =
    // R^q W^q (kind 2) in single bf16, for the contraction when the tiling
    // asks for one workgroup a CU.  bf16x3 U^q runs the two-stage pipeline
    // with two workgroups a CU whatever the tiling (1000-k shape, 14400 pair
    // rows: 0.127 against 0.119 of bf16 peak for the triangular factor
    // product, 0.146 against 0.141 for the full one; single bf16 0.274 on
    // the ring against 0.255).
    const bool ring = (prec == 2 || prec == 3) && ring_supported(conj, kind) &&
                      ((kind == 2 && prec == 3) || (kind == 3 && t_wg_per_cu == 1));
    const int blocks = ring ? max_gemm_blocks() / 8
                            : (prec == 2 && kind == 2 ? max_gemm_blocks() / 8 * 2 : gemm_blocks());
    HIPCHK(prec == 2   ? x3_launch(conj, dd, (int)d.size(), total, blocks, seg, s, kind, ring)
           : prec == 3 ? x1_launch(conj, dd, (int)d.size(), total, blocks, seg, s, kind, ring)
                       : big_launch(prec, conj, dd, (int)d.size(), total, gemm_blocks(), seg, s, kind));
    if (mark) mark(false);
  }
}

NtDesc mknt(const void* A, long long lda, const void* B, long long ldb, void* C, long long ldc,
            int M, int N, int K) {
  NtDesc d;
  memset(&d, 0, sizeof(d));
  d.A = A;
  d.B = B;
  d.C = C;
  d.lda = lda;
  d.ldb = ldb;
  d.ldc = ldc;
  d.M = M;
  d.N = N;
  d.Kseg = K;
  d.Klast = K;
  d.nseg = 1;
  d.batch = 1;
  return d;
}

// bytes per complex element of the GEMM operand format of a precision
size_t fmt_bytes(int prec) { return prec == 0 ? 16 : (prec == 3 ? 4 : 8); }
// bytes between consecutive elements of one row as addressed by pointers:
// c128, one FP32 plane (planes separate), bf16 hi/lo interleaved (8 bytes),
// single bf16 interleaved (4 bytes)
size_t fmt_scalar(int prec) { return prec == 0 ? 16 : (prec == 1 ? 4 : (prec == 2 ? 8 : 4)); }

GemmDesc mkdesc(const cplx* A, long long lda, const cplx* B, long long ldb, cplx* C, long long ldc,
                int M, int N, int K) {
  GemmDesc d;
  memset(&d, 0, sizeof(d));
  d.A = A;
  d.B = B;
  d.C = C;
  d.lda = lda;
  d.ldb = ldb;
  d.ldc = ldc;
  d.M = M;
  d.N = N;
  d.Kseg = K;
  d.Klast = K;
  d.nseg = 1;
  d.batch = 1;
  return d;
}

// Stage timer: pairs of HIP events recorded on the stream a stage runs on; a
// stage may be timed several times per call (e.g. once per grid tile) and the
// intervals are summed.
struct StageTimer {
  struct Slot {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
  };
  std::map<std::string, Slot> slots;
  std::map<std::string, float> ms;          // last call's sum
  void begin(const std::string& n, hipStream_t s) {
    Slot& sl = slots[n];
    if (sl.used == sl.ev.size()) {
      hipEvent_t a, b;
      HIPCHK(hipEventCreate(&a));
      HIPCHK(hipEventCreate(&b));
      sl.ev.emplace_back(a, b);
    }
    HIPCHK(hipEventRecord(sl.ev[sl.used].first, s));
  }
  void end(const std::string& n, hipStream_t s) {
    Slot& sl = slots[n];
    HIPCHK(hipEventRecord(sl.ev[sl.used].second, s));
    ++sl.used;
  }
  // After the stream has drained: sum the intervals recorded since the last
  // collect, and add them to totals (ms, count) if given.
  void collect(std::map<std::string, std::pair<double, long long>>* totals = nullptr) {
    for (auto& kv : slots) {
      Slot& sl = kv.second;
      if (sl.used == 0) continue;
      double sum = 0;
      for (size_t i = 0; i < sl.used; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, sl.ev[i].first, sl.ev[i].second) == hipSuccess) sum += t;
        else (void)hipGetLastError();
      }
      ms[kv.first] = (float)sum;
      if (totals) {
        (*totals)[kv.first].first += sum;
        (*totals)[kv.first].second += (long long)sl.used;
      }
      sl.used = 0;
    }
  }
  ~StageTimer() {
    for (auto& kv : slots)
      for (auto& e : kv.second.ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
  }
};

// One fragment of a batch.
struct FragIn {
  int nf;
  const void* C;
  void* eri;
  uint32_t flags;
};

// Workspace of one fragment batch (one in flight per workspace).
struct Workspace {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DevBuf mem;     // C_all | Tf | M | U | eri staging
  PinnedBuf hostc;  // staging for host C
  Arena arena;
  StageTimer timer;
  hipEvent_t done = nullptr;
  std::vector<uint64_t> tickets;
  std::vector<FragIn> frags;
  ~Workspace() {
    if (done) (void)hipEventDestroy(done);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

struct Request {
  isdf_request req;
  int state = ISDF_REQ_QUEUED;
  double t_submit = 0, t_done = 0;
  std::string err;
};

}  // namespace

struct isdf_ctx_s {
  // sizes
  int n[3], m[3];
  int nk = 0, norb = 0, nip = 0;
  long long ng = 0;
  double lattice[9], recip[9], volume = 0;
  uint32_t flags = 0;
  hipStream_t stream = nullptr;
  hipStream_t aux = nullptr;            // second stream: the factorisation overlaps the RHS
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_pinv = nullptr;
  // third stream: the RHS k convolution of one r tile beside the pre-product
  // of the next (two FP32 tiles in the tile buffer)
  hipStream_t aux2 = nullptr;
  hipEvent_t ev_rt[2] = {nullptr, nullptr}, ev_kc[2] = {nullptr, nullptr};
  int device = 0;
  // resident device data
  DevBuf phi, ip, xt, pi, eta, lt, w, work1, work2, work3, pinv_ws, perm, rank, rchunk, flag;
  DevBuf wt64, wt32, wt16, wt16s;       // W transposed in the four GEMM operand formats
  DevBuf dmax, cflag;                   // factorisation: largest diagonal, breakdown flags
  long long ld_ip = 0;                  // row pitch of the split operands (a multiple of 16)
  bool has_orbitals = false;            // false for a context restored by isdf_load
  bool fitted = false, kernel_ready = false, eta_valid = false;
  // the mixed operand copies hold sqrt(w_h) L^T (W^h = L L^H) instead of W^T:
  // U^q = R^q W^q becomes Y^q = R^q L^q and the contraction sum_q Y Y^H
  bool wfac = false;
  bool kernel_pending = false;          // a fit whose eta (resident or per batch) the kernel has not consumed
  bool etat_valid = false;              // eta~ of every class still held after the kernel (no q batches)
  // launch tiling of the fragment contraction (isdf_autotune / isdf_set_tiling):
  // classes per ERI launch (the K extent of one launch) and workgroups per CU
  // of its persistent GEMM launches (0: default)
  int eri_qgroup = ERI_QGROUP, frag_wg_per_cu = FRAG_WG_PER_CU;
  int eri_qgroup0 = ERI_QGROUP;         // the initial classes per launch (initial_qgroup of ld_ip)
  std::vector<int> rank_h;
  // q <-> -q: Pi^{-q}, W^{-q} and R^{-q}_{pq} are conjugates of those at q,
  // so the fragment contraction runs over the classes {q, -q}: hq[h] is the
  // smaller index of class h (nh classes), qslot[q] its class where q == hq,
  // else -1; hself[h] = 1 if q == -q.  Device copy qmap = [qslot | hq | hself].
  int nh = 0;
  std::vector<int> qslot_h, hq_h, hself_h;
  DevBuf qmap;
  // q batches: eta (and the split eta~, the factor table) hold qb classes at
  // a time; with qb < nh the RHS is formed per batch inside
  // isdf_coulomb_kernel instead of in isdf_fit (eta_batched)
  int qb = 0;
  bool eta_batched = false;
  long long rc = 0;   // RHS tile: rc grid points x ri interpolation points
  int ri = 0;
  Arena arena;
  Arena arena_aux;                      // descriptors of the second stream (chol, pinv)
  StageTimer timer;
  std::string err;
  // fragment workspace of the synchronous call
  Workspace sync_ws;
  // workspace of isdf_fragment_eri_static: attached to this device's copy of
  // the static scratch array (address from set-up), never allocated
  Workspace static_ws;
  void* scratch = nullptr;
  // serving
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool serving = false, stop = false;
  bool exclusive = false;               // a synchronous call holds the context (see Exclusive)
  int max_inflight = 2, max_batch = 64;
  long long budget = 0;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> queue;
  std::vector<Workspace*> ws_pool;
  long long served = 0, batches = 0;
  int inflight_n = 0;
  std::string serve_err;
  // accumulated device milliseconds and interval counts per stage
  std::map<std::string, std::pair<double, long long>> totals;
};

namespace {

// message of the last failed isdf_create on this thread (no context exists)
thread_local std::string t_create_err;

isdf_status fail(isdf_ctx c, isdf_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

template <class F> isdf_status guarded(isdf_ctx c, F&& f) {
  if (!c) return ISDF_E_INVALID;
  try {
    f();
    return ISDF_OK;
  } catch (const Fail& e) {
    c->err = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return ISDF_E_NOMEM;
  } catch (...) {
    c->err = "unexpected exception";
    return ISDF_E_INVALID;
  }
}

// Exclusive use of the context by a synchronous call that rewrites or times
// its GPU state (isdf_fit, isdf_coulomb_kernel, isdf_autotune,
// isdf_set_tiling): refused with ISDF_E_BUSY while served requests are queued
// or in flight (a batch counts from the moment its requests leave the queue);
// while it is held the serving thread admits nothing.  clear_kernel: W^q is
// invalid from the start of the call (a request admitted afterwards without
// a new kernel fails).
struct Exclusive {
  isdf_ctx c;
  Exclusive(isdf_ctx c_, bool clear_kernel) : c(c_) {
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->serving) {
      for (uint64_t t : c->queue) {
        auto it = c->reqs.find(t);
        if (it != c->reqs.end() && it->second.state == ISDF_REQ_QUEUED)
          throw Fail{ISDF_E_BUSY, "requests are queued or running"};
      }
      if (c->inflight_n != 0) throw Fail{ISDF_E_BUSY, "requests are queued or running"};
    }
    c->exclusive = true;
    if (clear_kernel) c->kernel_ready = false;
  }
  ~Exclusive() {
    std::lock_guard<std::mutex> lk(c->mu);
    c->exclusive = false;
    c->cv.notify_all();
  }
};

bool good_grid(int n) {
  if (n < 2 || n > 64) return false;
  int x = n;
  for (int f : {2, 3, 5, 7})
    while (x % f == 0) x /= f;
  return x == 1;
}

long long nip2(const isdf_ctx c) { return (long long)c->nip * c->nip; }

// --------------------------------------------------------------------------
// fit
// --------------------------------------------------------------------------
// eta^q_I(r) of the classes that qslot (device map q -> eta slot, or -1)
// selects, r-tiled: T^k_I(r) = sum_mu X^k_{I mu} conj(phi^k_mu(r)), then the
// k convolution of eq. (5) (Algorithm 1 with Y = phi), all in FP64.  Two tile
// buffers alternate, so the k convolution of tile i (third stream) runs
// beside the pre-product of tile i + 1.  The main stream continues after the
// last convolution; the third stream starts after `start` (recorded on the
// main stream).
void rhs_eta(isdf_ctx c, const int* qslot, hipEvent_t start) {
  hipStream_t s = c->stream;
  const int nk = c->nk, norb = c->norb, nip = c->nip;
  const long long ng = c->ng;
  constexpr int nbuf = 2;
  HIPCHK(hipStreamWaitEvent(c->aux2, start, 0));
  int it = 0;
  for (long long r0 = 0; r0 < ng; r0 += c->rc)
  for (int i0 = 0; i0 < nip; i0 += c->ri, ++it) {
    const int b = it % nbuf;
    cplx* tile = c->rchunk.as<cplx>() + (long long)b * nk * c->ri * c->rc;
    if (it >= nbuf) HIPCHK(hipStreamWaitEvent(s, c->ev_kc[b], 0));   // tile b read by its convolution
    c->timer.begin("rhs_t", s);
    const int rcur = (int)std::min<long long>(c->rc, ng - r0);
    const int icur = std::min(c->ri, nip - i0);
    HIPCHK(rhs_t_launch(c->xt.as<cplx>(), c->phi.as<cplx>(), tile, nk, norb, nip, ng, r0, rcur, i0, icur, s));
    c->timer.end("rhs_t", s);
    HIPCHK(hipEventRecord(c->ev_rt[b], s));
    HIPCHK(hipStreamWaitEvent(c->aux2, c->ev_rt[b], 0));
    c->timer.begin("rhs_kconv", c->aux2);
    KconvArgs a;
    memset(&a, 0, sizeof(a));
    a.in = tile;
    a.out = c->eta.as<cplx>() + (long long)i0 * ng + r0;
    a.in_kstride = (long long)icur * rcur;
    a.out_qstride = (long long)nip * ng;
    a.n_elem = (long long)icur * rcur;
    a.in_inner = a.n_elem;
    a.in_outer = 0;
    a.out_inner = rcur;
    a.out_outer = ng;
    a.m1 = c->m[0]; a.m2 = c->m[1]; a.m3 = c->m[2];
    a.mode = 0;
    a.scale = 1.0 / nk;
    a.qslot = qslot;                     // eta^{-q} = conj eta^q: one q per class
    HIPCHK(kconv_launch(a, c->aux2));
    c->timer.end("rhs_kconv", c->aux2);
    HIPCHK(hipEventRecord(c->ev_kc[b], c->aux2));
  }
  // eta complete: the main stream continues after the last convolution
  HIPCHK(hipStreamWaitEvent(s, c->ev_kc[(it - 1) % nbuf], 0));
}

// Buffers used only inside isdf_fit and isdf_coulomb_kernel: T^k of the
// metric and V per class (work1), the factorisation and pseudo-inverse
// scratch (lt, work2, work3, pinv_ws), the RHS tile and eta.  Allocated at
// create and again by a fit after a q-batched kernel released them.
void ensure_fit_buffers(isdf_ctx c) {
  const size_t e = sizeof(cplx);
  const size_t m2 = (size_t)c->nh * c->nip * c->nip * e;   // one matrix per class {q, -q}
  c->lt.ensure(m2);
  c->work1.ensure((size_t)c->nk * c->nip * c->nip * e);    // T^k of the metric, then V per class
  c->pinv_ws.ensure((size_t)c->nh * ((size_t)c->nip * 64 + 4096) * e);   // blocked L^{-1} scratch
  c->work2.ensure(m2);
  c->work3.ensure(m2);
  c->rchunk.ensure(2 * (size_t)c->nk * c->ri * c->rc * e);   // two RHS tiles
  c->eta.ensure((size_t)c->qb * c->nip * c->ng * e);
}

// After a kernel that ran in q batches (memory-bound cells), the transient
// buffers go back to the device for the fragment workspaces; X, Pi^q, W^q
// and its operand copies stay.
void release_fit_buffers(isdf_ctx c) {
  for (DevBuf* b : {&c->lt, &c->work1, &c->pinv_ws, &c->work2, &c->work3, &c->rchunk, &c->eta})
    b->release();
}

// Workspace bytes of one served batch.
long long serve_cap(isdf_ctx c) { return c->budget / c->max_inflight; }

// Serving workspaces sized to their share of the budget (idle ones only:
// called at isdf_serve_start and after a Coulomb kernel, under exclusive use).
void reserve_workspaces(isdf_ctx c) {
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->serving && c->ws_pool.empty()) return;
  for (Workspace* w : c->ws_pool) w->mem.ensure((size_t)serve_cap(c));
}

// The fit reclaims the memory of idle fragment workspaces (the context is
// held exclusively: no batch is in flight).
void release_workspaces(isdf_ctx c) {
  HIPCHK(hipStreamSynchronize(c->stream));
  c->sync_ws.mem.release();
  std::lock_guard<std::mutex> lk(c->mu);
  for (Workspace* w : c->ws_pool) w->mem.release();
}

// Blocked right-looking Cholesky of nq Hermitian n x n matrices at once
// (64-wide diagonal blocks in LDS, panel solves, FP64 MFMA trailing
// updates), no pivoting: the factor in the lower triangle of A and, transposed,
// in lt; flag[q] set where a pivot is not above rtol * max diagonal.
void chol_blocked(Arena& ar, const cplx* in, cplx* A, cplx* lt, int* perm, int* rank, double* dmax, int* flag, int n,
                  int nq, double rtol, hipStream_t s) {
  const long long nn = (long long)n * n;
  HIPCHK(bchol_setup_launch(in, A, perm, rank, dmax, flag, n, nq, s));
  for (int jb = 0; jb < n; jb += CHOL_NB) {
    HIPCHK(bchol_diag_launch(A, lt, dmax, flag, n, nq, jb, rtol, s));
    HIPCHK(bchol_panel_launch(A, lt, flag, n, nq, jb, s));
    const int rest = n - jb - CHOL_NB;
    if (rest > 0) {
      std::vector<NtDesc> d(1);
      const cplx* L21 = A + (long long)(jb + CHOL_NB) * n + jb;
      d[0] = mknt(L21, n, L21, n, A + (long long)(jb + CHOL_NB) * (n + 1), n, rest, rest, CHOL_NB);
      d[0].batch = nq;
      d[0].sA_bat = d[0].sB_bat = d[0].sC_bat = nn;
      d[0].herm = 2;
      d[0].epi = 4;
      run_nt(ar, 0, 2, d, s);
    }
  }
}

void do_fit(isdf_ctx c, int prec) {
  hipStream_t s = c->stream;
  const int nk = c->nk, norb = c->norb, nip = c->nip;
  const int nh = c->nh;                 // classes {q, -q}: Pi, eta, W are kept for one q of each
  const long long ng = c->ng;
  if (!c->eta.p) {
    release_workspaces(c);
    ensure_fit_buffers(c);
  }
  c->arena.reset(s);
  c->arena.reserve(((size_t)1 << 20) + (size_t)c->nh * 1024);
  // the second stream may still be forming the previous fit's pseudo-inverse
  c->arena_aux.reset(c->aux);
  c->arena_aux.reserve(((size_t)1 << 20) + (size_t)c->nh * 1024);
  // X^k (IV gather)
  HIPCHK(gather_launch(c->phi.as<cplx>(), c->ip.as<int>(), c->xt.as<cplx>(), nk, norb, ng, nip, s));
  // T^k_IJ = sum_mu X^k_{I mu} conj(X^k_{J mu})  (Algorithm 1, Y = X)
  c->timer.begin("metric_t", s);
  {
    std::vector<GemmDesc> d(1);
    d[0] = mkdesc(c->xt.as<cplx>(), nip, c->xt.as<cplx>(), nip, c->work1.as<cplx>(), nip, nip, nip, norb);
    d[0].batch = nk;
    d[0].sA_bat = d[0].sB_bat = (long long)norb * nip;
    d[0].sC_bat = nip2(c);
    d[0].herm = 1;
    run_gemm(c->arena, 0, GEMM_A_KM | GEMM_B_KN | GEMM_B_CONJ, d, s);
  }
  c->timer.end("metric_t", s);
  // Pi^q = N_k^-1 sum_R exp(iq.R) |sum_k exp(ik.R) T^k|^2   (eq. (4), Algorithm 1),
  // kept for one q per class (Pi^{-q} = conj Pi^q), in class order
  c->timer.begin("metric_kconv", s);
  {
    KconvArgs a;
    memset(&a, 0, sizeof(a));
    a.in = c->work1.as<cplx>();
    a.out = c->pi.as<cplx>();
    a.in_kstride = a.out_qstride = nip2(c);
    a.n_elem = nip2(c);
    a.in_inner = a.out_inner = a.n_elem;
    a.in_outer = a.out_outer = 0;
    a.m1 = c->m[0]; a.m2 = c->m[1]; a.m3 = c->m[2];
    a.mode = 0;
    a.scale = 1.0 / nk;
    a.qslot = c->qmap.as<int>();
    HIPCHK(kconv_launch(a, s));
  }
  c->timer.end("metric_kconv", s);
  // FP64 pivoted Cholesky of every Pi^q (solve of eq. (3)) on the second
  // stream, overlapping the RHS below (it needs only Pi)
  HIPCHK(hipEventRecord(c->ev_fork, s));
  HIPCHK(hipStreamWaitEvent(c->aux, c->ev_fork, 0));
  // eta^q_I(r) for every class now when they all fit (else per q batch in
  // isdf_coulomb_kernel)
  (void)prec;
  c->eta_batched = c->qb < nh;
  if (!c->eta_batched) rhs_eta(c, c->qmap.as<int>(), c->ev_fork);
  c->timer.begin("chol", c->aux);
  {
    // blocked right-looking factorisation of all Pi^q at once: 64-wide
    // diagonal blocks in LDS, panel solves, FP64 MFMA trailing updates
    cplx* A = c->work2.as<cplx>();
    const double rtol = 1e-13;
    chol_blocked(c->arena_aux, c->pi.as<cplx>(), A, c->lt.as<cplx>(), c->perm.as<int>(), c->rank.as<int>(),
                 c->dmax.as<double>(), c->cflag.as<int>(), nip, nh, rtol, c->aux);
    // matrices whose pivots fell below the rank tolerance (singular metrics)
    // are refactored with diagonal pivoting
    std::vector<int> fl(nh, 0);
    HIPCHK(hipMemcpyAsync(fl.data(), c->cflag.p, sizeof(int) * nh, hipMemcpyDeviceToHost, c->aux));
    HIPCHK(hipStreamSynchronize(c->aux));
    std::vector<int> qs;
    for (int h = 0; h < nh; ++h)
      if (fl[h]) qs.push_back(h);
    if (!qs.empty()) {
      int* ql = c->arena_aux.put(qs.data(), qs.size(), c->aux);
      HIPCHK(chol_launch(c->pi.as<cplx>(), A, c->lt.as<cplx>(), c->perm.as<int>(), c->rank.as<int>(),
                         nip, (int)qs.size(), rtol, (c->flags & ISDF_NO_PIVOT) ? 0 : 1, c->aux, ql));
    }
  }
  c->timer.end("chol", c->aux);
  HIPCHK(hipEventRecord(c->ev_join, c->aux));
  HIPCHK(hipStreamWaitEvent(s, c->ev_join, 0));
  c->rank_h.assign(nh, 0);
  HIPCHK(hipMemcpyAsync(c->rank_h.data(), c->rank.p, sizeof(int) * nh, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->timer.collect(&c->totals);
  }
  for (int h = 0; h < nh; ++h) {
    const int q = c->hq_h[h];
    if (c->rank_h[h] <= 0)
      throw Fail{ISDF_E_NUMERIC, "metric Pi^q is zero or not finite at q = " + std::to_string(q)};
    if ((c->flags & ISDF_NO_PIVOT) && c->rank_h[h] < nip)
      throw Fail{ISDF_E_NUMERIC, "Cholesky breakdown of Pi^q (singular metric) at q = " + std::to_string(q) +
                                     ", column " + std::to_string(c->rank_h[h])};
  }
  // The pseudo-inverse factor of eq. (8) on the second stream: it overlaps
  // the grid FFT and the V^q product of isdf_coulomb_kernel, which waits for
  // it (ev_pinv) before W^q = G V' G.
  c->timer.begin("pinv", c->aux);
  {
    cplx* A = c->work2.as<cplx>();
    // Y = L^{-1} by 64-row block rows (zero outside the rank block; stored
    // transposed in A = work2), G = Y^H Y (into work3), so that
    // P^T Pi^+ P = G on the rank block.  Scratch: the row-major factor in
    // work3 (overwritten by G at the end), the block-row partials St [n][64]
    // and the diagonal inverses in pinv_ws.
    {
      cplx* Lrow = c->work3.as<cplx>();
      cplx* St = c->pinv_ws.as<cplx>();
      cplx* Yd = St + (long long)nh * nip * 64;
      const long long nn = nip2(c);
      HIPCHK(tri_setup_launch(c->lt.as<cplx>(), c->rank.as<int>(), Lrow, A, nip, nh, c->aux));
      for (int jb = 0; jb < nip; jb += 64) {
        const int nb = std::min(64, nip - jb);
        if (jb > 0) {
          // St[n][m] = sum_{k < jb} Yt[n][k] L[jb+m][k]
          std::vector<NtDesc> g(1);
          g[0] = mknt(A, nip, Lrow + (long long)jb * nip, nip, St, 64, jb, nb, jb);
          g[0].batch = nh;
          g[0].sA_bat = g[0].sB_bat = nn;
          g[0].sC_bat = (long long)nip * 64;
          run_nt(c->arena_aux, 0, 0, g, c->aux);
        }
        HIPCHK(tri_inv_diag_launch(Lrow, c->rank.as<int>(), A, Yd, nip, nh, jb, c->aux));
        if (jb > 0) {
          // Yt[n][jb+m] = Y[jb+m][n] = -sum_k St[n][k] Y_bb[m][k]
          std::vector<NtDesc> g(1);
          g[0] = mknt(St, 64, Yd, 64, A + jb, nip, jb, nb, nb);
          g[0].batch = nh;
          g[0].sA_bat = (long long)nip * 64;
          g[0].sB_bat = 4096;
          g[0].sC_bat = nn;
          g[0].epi = 4;
          run_nt(c->arena_aux, 0, 0, g, c->aux);
        }
      }
    }
    std::vector<NtDesc> d(1);
    d[0] = mknt(A, nip, A, nip, c->work3.as<cplx>(), nip, nip, nip, nip);
    d[0].batch = nh;
    d[0].sA_bat = d[0].sB_bat = d[0].sC_bat = nip2(c);
    d[0].herm = 1;
    // G[m][n] = sum_i conj(Yt[m][i]) Yt[n][i]
    run_nt(c->arena_aux, 0, 1, d, c->aux);
  }
  c->timer.end("pinv", c->aux);
  HIPCHK(hipEventRecord(c->ev_pinv, c->aux));
  c->fitted = true;
  c->eta_valid = !c->eta_batched;
  c->kernel_pending = true;
  c->kernel_ready = false;
}

// --------------------------------------------------------------------------
// Coulomb kernel
// --------------------------------------------------------------------------
// The fragment GEMMs' operands from W^q: transposed copies in the four
// formats (one per class {q, -q}, weight 1/2 where q = -q: the fragment
// contraction adds the conjugate term of -q itself).  Then every W^h (FP64,
// Hermitian positive semidefinite) is factored W^h = L L^H without pivoting;
// when every pivot is above WFAC_RTOL times the largest diagonal entry of its
// matrix, the mixed copies take sqrt(w_h) L^T instead, so that U^q = R^q W^q
// becomes the triangular product Y^q = R^q L^q (half the work) and the
// contraction sum_q U R^H becomes sum_q Y Y^H.  Otherwise (a singular or
// too ill-conditioned W^h: a rank-deficient metric) the copies stay W^T.
// work, lt: two [nh][n][n] c128 buffers, or null (allocated here).
constexpr double WFAC_RTOL = 1e-13;
void operand_copies(isdf_ctx c, cplx* work, cplx* lt, hipStream_t s) {
  const int nk = c->nk, nip = c->nip, nh = c->nh;
  const int* hself = c->qmap.as<int>() + nk + nh;
  HIPCHK(wt_convert_launch(c->w.as<cplx>(), c->wt64.as<cplx>(), c->wt32.as<float>(), c->wt16.as<unsigned short>(),
                           c->wt16s.as<unsigned short>(), nip, (int)c->ld_ip, nh, hself, s));
  c->wfac = false;
  if (c->flags & ISDF_W_PLAIN) {
    HIPCHK(hipStreamSynchronize(s));
    return;
  }
  const size_t m2 = (size_t)nh * nip * nip * sizeof(cplx);
  DevBuf wa, wl, perm, rank, dmax, flag;
  try {
    if (!work) { wa.alloc(m2); work = wa.as<cplx>(); }
    if (!lt) { wl.alloc(m2); lt = wl.as<cplx>(); }
    perm.alloc(sizeof(int) * nh * (size_t)nip);
    rank.alloc(sizeof(int) * nh);
    dmax.alloc(sizeof(double) * nh);
    flag.alloc(sizeof(int) * nh);
  } catch (const Fail&) {
    (void)hipGetLastError();
    return;                               // no room for the factor: W^T copies
  }
  chol_blocked(c->arena, c->w.as<cplx>(), work, lt, perm.as<int>(), rank.as<int>(), dmax.as<double>(),
               flag.as<int>(), nip, nh, WFAC_RTOL, s);
  std::vector<int> fl(nh);
  HIPCHK(hipMemcpyAsync(fl.data(), flag.p, sizeof(int) * nh, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int f : fl)
    if (f) return;
  HIPCHK(lt_convert_launch(lt, c->wt32.as<float>(), c->wt16.as<unsigned short>(), c->wt16s.as<unsigned short>(), nip,
                           (int)c->ld_ip, nh, hself, s));
  HIPCHK(hipStreamSynchronize(s));
  c->wfac = true;
}

// Common end of both routes: W^q in the fragment GEMMs' operand formats, the
// finiteness check, and the fit's transient buffers handed back.
void kernel_finish(isdf_ctx c) {
  hipStream_t s = c->stream;
  const int nk = c->nk, nip = c->nip, nh = c->nh;
  HIPCHK(hipMemsetAsync(c->flag.p, 0, sizeof(int), s));
  HIPCHK(nonfinite_launch(c->w.as<cplx>(), (long long)nh * nip2(c), c->flag.as<int>(), s));
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (!bad) {
    // the factorisation scratch of the fit, when it is there
    const size_t m2 = (size_t)nh * nip * nip * sizeof(cplx);
    operand_copies(c, c->work2.bytes >= m2 ? c->work2.as<cplx>() : nullptr,
                   c->work3.bytes >= m2 ? c->work3.as<cplx>() : nullptr, s);
  }
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->timer.collect(&c->totals);
  }
  if (bad) throw Fail{ISDF_E_NUMERIC, "non-finite entries in W^q"};
  if (c->eta_batched) {
    release_fit_buffers(c);
    try {
      reserve_workspaces(c);
    } catch (const Fail&) {
      // the serving workspaces then grow when a batch needs them
    }
  }
  c->kernel_ready = true;
}

// The zeta route (eqs. (3), (6)), all FP64:
//   xi^q = Pi^{q+} eta^q  with Pi^{q+} = P G P^T (G = L^{-H} L^{-1} on the rank
//   block of the pivoted factor, formed by isdf_fit), one MFMA product
//   [N_IP x N_IP] [N_IP x N_g] per class;
//   xi~^q_I(G) = sqrt(Omega 4pi/|K|^2)/N_g FFT[xi^q_I(r) exp(-iq.r)], in place;
//   W^q = xi~ xi~^H (lower tiles, mirrored).
// eta is left in place (it stays valid); xi lives in a buffer of eta's size
// that is freed on return.
void kernel_zeta_route(isdf_ctx c) {
  hipStream_t s = c->stream;
  const int nip = c->nip, nh = c->nh, nk = c->nk;
  const long long ng = c->ng;
  if (c->eta_batched || !c->eta_valid)
    throw Fail{ISDF_E_NOMEM, "the zeta route needs eta of every class resident (isdf_fit formed it per q batch)"};
  DevBuf xi;
  xi.alloc(sizeof(cplx) * (size_t)nh * nip * ng);
  HIPCHK(hipStreamWaitEvent(s, c->ev_pinv, 0));   // G from isdf_fit's second stream
  c->timer.begin("zeta_solve", s);
  {
    // Pi^+ in natural order (zero outside the rank block before the scatter)
    HIPCHK(permute_launch(c->work3.as<cplx>(), c->work2.as<cplx>(), c->perm.as<int>(), c->rank.as<int>(), nip, nh,
                          1, s));
    std::vector<GemmDesc> d(1);
    d[0] = mkdesc(c->work2.as<cplx>(), nip, c->eta.as<cplx>(), ng, xi.as<cplx>(), ng, nip, (int)ng, nip);
    d[0].batch = nh;
    d[0].sA_bat = nip2(c);
    d[0].sB_bat = d[0].sC_bat = (long long)nip * ng;
    run_gemm(c->arena, 0, GEMM_B_KN, d, s);
  }
  c->timer.end("zeta_solve", s);
  c->timer.begin("grid_fft", s);
  {
    GridFftArgs a;
    memset(&a, 0, sizeof(a));
    a.data = xi.as<cplx>();
    a.n1 = c->n[0]; a.n2 = c->n[1]; a.n3 = c->n[2];
    a.m1 = c->m[0]; a.m2 = c->m[1]; a.m3 = c->m[2];
    a.q0 = 0;
    a.nq = nh;
    a.qlist = c->qmap.as<int>() + nk;
    a.n_ip = nip;
    a.q_stride = (long long)nip * ng;
    memcpy(a.recip, c->recip, sizeof(a.recip));
    a.volume = c->volume;
    HIPCHK(gridfft_launch(a, s));
  }
  c->timer.end("grid_fft", s);
  c->timer.begin("w_gemm", s);
  {
    std::vector<NtDesc> d(1);
    d[0] = mknt(xi.p, ng, xi.p, ng, c->w.p, nip, nip, nip, (int)ng);
    d[0].sA_bat = d[0].sB_bat = (long long)nip * ng;
    d[0].batch = nh;
    d[0].sC_bat = nip2(c);
    d[0].herm = 1;
    run_nt(c->arena, ISDF_FP64, 2, d, s, 1);
  }
  c->timer.end("w_gemm", s);
  c->kernel_pending = false;
  c->etat_valid = false;
  kernel_finish(c);
  // xi is freed with its buffer once the stream has drained (kernel_finish
  // synchronised it)
}

void do_kernel(isdf_ctx c, int prec) {
  if (!c->fitted || !c->kernel_pending) throw Fail{ISDF_E_STATE, "isdf_fit must run before isdf_coulomb_kernel"};
  // The kernel is FP64 in every precision: W^q = Pi^+ V^q Pi^+ amplifies the
  // rounding of eta and V^q by up to cond(Pi^q) on each side, and at the
  // conditioning of the workloads (1e4-5e5) FP32 or bf16 hi+lo eta / V^q move
  // the ERIs by 3e-6-2e-5 Eh.  The mixed precisions apply to the fragment
  // GEMMs, whose error with an FP64 W^q stays far smaller.
  (void)prec;
  hipStream_t s = c->stream;
  const int nk = c->nk, nip = c->nip;
  const int nh = c->nh;                 // one q per class {q, -q}: W^{-q} = conj W^q
  const long long ng = c->ng;
  c->arena.reset(s);
  // per q batch: the slot map and a few descriptors; the W solve: one
  // descriptor per class for each of its two products
  c->arena.reserve(((size_t)1 << 20) + (size_t)nh * 2 * (sizeof(NtDesc) + 256) +
                   (size_t)((nh + std::max(c->qb, 1) - 1) / std::max(c->qb, 1)) * (nk * sizeof(int) + 4096));
  // the zeta route of eqs. (3) and (6): xi^q = Pi^{q+} eta^q, FFT, W^q = xi~ xi~^H
  if (c->flags & ISDF_ZETA_ROUTE) {
    kernel_zeta_route(c);
    return;
  }
  // q batches of qb classes (one batch, eta formed by the fit, when they all
  // fit); per batch: eta (when batched), the grid FFT, V^q
  const int qb = c->eta_batched ? c->qb : nh;
  std::vector<int> bslot(nk);
  for (int h0 = 0; h0 < nh; h0 += qb) {
    const int nb = std::min(qb, nh - h0);
    if (c->eta_batched) {
      // eta of classes h0 .. h0 + nb - 1 into slots 0 .. nb - 1 (eq. (5))
      for (int q = 0; q < nk; ++q) {
        const int h = c->qslot_h[q];
        bslot[q] = (h >= h0 && h < h0 + nb) ? h - h0 : -1;
      }
      const int* bs = c->arena.put(bslot.data(), bslot.size(), s);
      HIPCHK(hipEventRecord(c->ev_fork, s));   // the previous batch's FFT has read eta
      rhs_eta(c, bs, c->ev_fork);
    }
    // eta~^q_I(G) = sqrt(Omega 4pi/|K|^2)/N_g FFT[eta^q_I(r) exp(-iq.r)]   (eqs. (6)-(7)), in place
    c->timer.begin("grid_fft", s);
    {
      GridFftArgs a;
      memset(&a, 0, sizeof(a));
      a.data = c->eta.as<cplx>();
      a.n1 = c->n[0]; a.n2 = c->n[1]; a.n3 = c->n[2];
      a.m1 = c->m[0]; a.m2 = c->m[1]; a.m3 = c->m[2];
      a.q0 = 0;
      a.nq = nb;
      a.qlist = c->qmap.as<int>() + nk + h0;
      a.n_ip = nip;
      a.q_stride = (long long)nip * ng;
      memcpy(a.recip, c->recip, sizeof(a.recip));
      a.volume = c->volume;
      HIPCHK(gridfft_launch(a, s));
    }
    c->timer.end("grid_fft", s);
    // V^q = eta~ eta~^H  (Hermitian; lower tiles computed and mirrored), FP64 MFMA
    c->timer.begin("v_gemm", s);
    {
      cplx* vout = c->work1.as<cplx>() + (long long)h0 * nip2(c);
      std::vector<NtDesc> d(1);
      d[0] = mknt(c->eta.p, ng, c->eta.p, ng, vout, nip, nip, nip, (int)ng);
      d[0].sA_bat = d[0].sB_bat = (long long)nip * ng;
      d[0].batch = nb;
      d[0].sC_bat = nip2(c);
      d[0].herm = 1;
      run_nt(c->arena, ISDF_FP64, 2, d, s, 1);
    }
    c->timer.end("v_gemm", s);
  }
  c->eta_valid = false;
  c->kernel_pending = false;
  c->etat_valid = !c->eta_batched;
  // W^q = Pi^{q+} V^q Pi^{q+}   (eq. (8)) in FP64 through the pivoted factor
  // P^T Pi P = L L^H of rank r:  G = L^{-H} L^{-1} (formed by isdf_fit),
  // W' = G (P^T V P) G, W = P W' P^T (zero outside the rank block); the two
  // products are FP64 MFMA.
  HIPCHK(hipStreamWaitEvent(s, c->ev_pinv, 0));   // G from isdf_fit's second stream
  c->timer.begin("w_solve", s);
  {
    const long long n2 = nip2(c);
    HIPCHK(permute_launch(c->work1.as<cplx>(), c->w.as<cplx>(), c->perm.as<int>(), c->rank.as<int>(),
                          nip, nh, 0, s));
    auto prod = [&](const cplx* A, const cplx* B, cplx* C, int conj, int herm) {
      std::vector<NtDesc> d;
      for (int h = 0; h < nh; ++h) {
        const int r = c->rank_h[h];
        NtDesc g = mknt(A + h * n2, nip, B + h * n2, nip, C + h * n2, nip, r, r, r);
        g.herm = herm;
        d.push_back(g);
      }
      run_nt(c->arena, 0, conj, d, s);
    };
    // T1 = G V'  (V' Hermitian: V'[k][n] = conj(V'[n][k]))
    prod(c->work3.as<cplx>(), c->w.as<cplx>(), c->work1.as<cplx>(), 2, 0);
    // W' = T1 G  (G Hermitian); W' = G V' G is Hermitian: lower tiles, mirrored
    prod(c->work1.as<cplx>(), c->work3.as<cplx>(), c->work2.as<cplx>(), 2, 1);
    HIPCHK(permute_launch(c->work2.as<cplx>(), c->w.as<cplx>(), c->perm.as<int>(), c->rank.as<int>(),
                          nip, nh, 1, s));
  }
  c->timer.end("w_solve", s);
  kernel_finish(c);
}

// --------------------------------------------------------------------------
// fragment ERIs
// --------------------------------------------------------------------------
struct BatchPlan {
  int ncol = 0;
  long long ptot = 0;
  std::vector<int> col, nf;
  std::vector<long long> poff, eoff;
  std::vector<long long> aoff;   // per fragment offset in the FP64 accumulation region
  // (pq)-blocking of the single fragment of a blocked batch: its nf^2 pairs
  // in nb blocks of at most pb pairs; R^q of two blocks (row block i and
  // column block j) and U^q of block i are held at a time
  int nb = 1;
  long long pb = 0;
  bool psi32 = false;            // the register pair transform reads psi as complex FP32
  size_t off_c = 0, off_tf = 0, off_psi = 0, off_m = 0, off_m2 = 0, off_u = 0, off_e = 0, off_acc = 0,
         bytes = 0;
  size_t arena_bytes = 0;        // descriptor bytes of the whole pass (upper bound)
};

constexpr int MAX_PAIR_BLOCKS = 32;

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Layout of one fragment batch in its workspace:
//   C_all [N_k][n_orb][ncol] c128          coefficients of all fragments
//   Tf    [N_k][ncol][N_IP] c128           T^k_{Ip} = sum_mu X C, then psi(r_I + R)
//   psi32 [N_k][ncol][N_IP] complex FP32   psi for the register pair transform
//                                          (blocked batches; otherwise staged in U)
//   M     [rows][nh][ld_ip] (format)       R^q_{I,pq} for one q of each class {q, -q},
//                                          rows = pairs of all fragments (or of block i)
//   M2    [pb][nh][ld_ip] (format)         R^q of column block j (blocked batches)
//   U     [rows][nh][ld_ip] (format)       U^q = R^q W^q (also stages host C first)
//   E     host-bound ERI outputs (c128)
//   acc   FP64 G_f[(pq)][(sr)] of every fragment
// nb == 1: every fragment unblocked; nb > 1: one fragment, pairs in nb blocks.
BatchPlan plan_batch(isdf_ctx c, const std::vector<FragIn>& fr, int prec, int nb) {
  BatchPlan p;
  long long ecount = 0, acount = 0;
  for (const FragIn& f : fr) {
    p.col.push_back(p.ncol);
    p.nf.push_back(f.nf);
    p.poff.push_back(p.ptot);
    p.ncol += f.nf;
    p.ptot += (long long)f.nf * f.nf;
    const long long e4 = (long long)f.nf * f.nf * f.nf * f.nf;
    p.eoff.push_back((f.flags & ISDF_FRAG_DEVICE) ? -1 : ecount);
    if (!(f.flags & ISDF_FRAG_DEVICE)) ecount += e4;
    p.aoff.push_back(acount);
    acount += e4;
  }
  p.nb = std::max(1, nb);
  p.pb = (p.ptot + p.nb - 1) / p.nb;
  // the mixed precisions' pair transforms read psi as complex FP32
  p.psi32 = prec != 0;
  const size_t row = (size_t)c->nh * c->ld_ip * fmt_bytes(prec);   // one pair row of R^q / U^q
  const size_t rows = p.nb == 1 ? (size_t)p.ptot : (size_t)p.pb;
  const size_t cstage = (size_t)c->nk * c->norb * p.ncol * sizeof(cplx);
  const size_t psi32b = (size_t)c->nk * p.ncol * c->nip * sizeof(float2);
  size_t off = 0;
  p.off_c = off; off += al256(cstage);
  p.off_tf = off; off += al256((size_t)c->nk * c->nip * p.ncol * sizeof(cplx));
  if (p.nb > 1 && p.psi32) { p.off_psi = off; off += al256(psi32b); }
  p.off_m = off; off += al256(rows * row);
  if (p.nb > 1) { p.off_m2 = off; off += al256(rows * row); }
  p.off_u = off;
  if (p.nb == 1 || !p.psi32) p.off_psi = off;   // psi32 staged in U until U^q is formed
  off += al256(std::max(rows * row, std::max(cstage, p.psi32 && p.nb == 1 ? psi32b : (size_t)0)));
  p.off_e = off; off += al256((size_t)ecount * sizeof(cplx));
  p.off_acc = off; off += al256((size_t)acount * sizeof(cplx));
  p.bytes = off;
  // descriptor arena: per-fragment tables, the pair blocks of every pair
  // transform table set (one per pair block), the GEMM descriptors (one per
  // fragment, or one per block pair), 256 bytes of alignment per put
  const size_t nfr = fr.size();
  const size_t ntab = (size_t)p.nb;
  const size_t nblk_pairs = (size_t)p.ptot + ntab * nfr;          // PairBlocks at tp = 1 (upper bound)
  p.arena_bytes = 256 * (size_t)(64 + 16 * ntab) + nblk_pairs * sizeof(PairBlock) +
                  ntab * (nfr * 48 + 64) + (nfr + 8) * 64 +
                  ((size_t)p.nb * (p.nb + 1) / 2 + nfr + 8) * (sizeof(NtDesc) + 256) + 4 * sizeof(GemmDesc);
  return p;
}

// Device bytes of one fragment batch's workspace (no allocation).
size_t batch_bytes(isdf_ctx c, const std::vector<FragIn>& fr, int prec, int nb) {
  return plan_batch(c, fr, prec, nb).bytes;
}

// Smallest pair-block count (1 = unblocked) whose workspace for the single
// fragment `f` fits `cap` bytes, or 0 if none up to MAX_PAIR_BLOCKS does.
int blocks_for(isdf_ctx c, const FragIn& f, int prec, size_t cap) {
  std::vector<FragIn> one(1, f);
  const long long np = (long long)f.nf * f.nf;
  for (int nb = 1; nb <= MAX_PAIR_BLOCKS && nb <= np; ++nb)
    if (batch_bytes(c, one, prec, nb) <= cap) return nb;
  return 0;
}

// Workspace bytes a request needs at least (at the largest pair blocking).
size_t request_bytes(isdf_ctx c, int nf, bool host_out, int prec) {
  FragIn f{nf, nullptr, nullptr, host_out ? 0u : (uint32_t)ISDF_FRAG_DEVICE};
  std::vector<FragIn> one(1, f);
  const long long np = (long long)nf * nf;
  return batch_bytes(c, one, prec, (int)std::min<long long>(MAX_PAIR_BLOCKS, np));
}

// Device tables of one pair transform over pair range [p0, p0 + np) of each
// fragment of the batch (np = all pairs when the batch is unblocked).
struct PairTables {
  const PairBlock* blocks = nullptr;
  const long long* item_off = nullptr;
  const long long* frag_pair = nullptr;
  const int* frag_p0 = nullptr;
  const int* frag_np = nullptr;
  int nblocks = 0;
  long long nitems = 0;
};

// Enqueue the whole fragment pipeline of one batch on ws.stream.  capture:
// the stream is being captured into a graph (no synchronisation; the
// workspace and arena were sized by an eager pass).
void enqueue_batch(isdf_ctx c, Workspace& ws, int prec, const std::vector<FragIn>& fr, bool timed,
                   int nb = 1, bool capture = false) {
  if (!c->kernel_ready) throw Fail{ISDF_E_STATE, "isdf_coulomb_kernel must run before fragment ERIs"};
  if (nb > 1 && fr.size() != 1) throw Fail{ISDF_E_INVALID, "pair blocking applies to one fragment"};
  hipStream_t s = ws.stream;
  WgScope wg(c->frag_wg_per_cu);
  const int nk = c->nk, norb = c->norb, nip = c->nip;
  const long long ld = c->ld_ip;
  BatchPlan p = plan_batch(c, fr, prec, nb);
  if (!capture) {
    ws.arena.reset(s);
    ws.arena.reserve(p.arena_bytes);
    ws.mem.ensure(p.bytes);
  } else {
    if (p.bytes > ws.mem.bytes) throw Fail{ISDF_E_INVALID, "captured batch larger than its workspace"};
    ws.arena.used = 0;
  }
  char* base = ws.mem.as<char>();
  cplx* Call = (cplx*)(base + p.off_c);
  cplx* Tf = (cplx*)(base + p.off_tf);
  char* Mq = base + p.off_m;
  char* Mq2 = base + p.off_m2;
  char* Uq = base + p.off_u;
  float2* psi32 = (float2*)(base + p.off_psi);
  cplx* Est = (cplx*)(base + p.off_e);
  cplx* acc = (cplx*)(base + p.off_acc);
  // upload / gather the fragment coefficients into C_all[k][mu][col]
  size_t host_bytes = 0;
  for (const FragIn& f : fr)
    if (!(f.flags & ISDF_FRAG_DEVICE)) host_bytes += (size_t)nk * norb * f.nf * sizeof(cplx);
  if (host_bytes) ws.hostc.ensure(host_bytes);
  // the staged host copies land in the U region first (free until step 13)
  size_t hoff = 0;
  std::vector<const cplx*> srcs(fr.size());
  int maxnf = 0;
  for (size_t i = 0; i < fr.size(); ++i) {
    const FragIn& f = fr[i];
    const size_t fb = (size_t)nk * norb * f.nf * sizeof(cplx);
    srcs[i] = (const cplx*)f.C;
    if (!(f.flags & ISDF_FRAG_DEVICE)) {
      memcpy((char*)ws.hostc.p + hoff, f.C, fb);
      HIPCHK(hipMemcpyAsync(Uq + hoff, (char*)ws.hostc.p + hoff, fb, hipMemcpyHostToDevice, s));
      srcs[i] = (const cplx*)(Uq + hoff);
      hoff += fb;
    }
    maxnf = std::max(maxnf, f.nf);
  }
  HIPCHK(copy_cols_batch_launch(ws.arena.put(srcs.data(), srcs.size(), s), Call, nk, norb,
                                ws.arena.put(p.nf.data(), p.nf.size(), s),
                                ws.arena.put(p.col.data(), p.col.size(), s), (int)fr.size(), maxnf, p.ncol, s));
  if (timed) ws.timer.begin("frag_t", s);
  // T^k_{pI} = sum_mu C^k_{mu p} X^k_{I mu}   (Algorithm 2, stored [k][p][I])
  {
    std::vector<GemmDesc> d(1);
    d[0] = mkdesc(Call, p.ncol, c->xt.as<cplx>(), nip, Tf, nip, p.ncol, nip, norb);
    d[0].batch = nk;
    d[0].sA_bat = (long long)norb * p.ncol;
    d[0].sB_bat = (long long)norb * nip;
    d[0].sC_bat = (long long)nip * p.ncol;
    run_gemm(ws.arena, 0, GEMM_A_KM | GEMM_B_KN, d, s);
  }
  // psi_p(r_I + R) = N_k^{-1/2} sum_k exp(ik.R) T^k_{pI}
  {
    KconvArgs a;
    memset(&a, 0, sizeof(a));
    a.in = Tf;
    a.out = Tf;
    a.in_kstride = a.out_qstride = (long long)nip * p.ncol;
    a.n_elem = (long long)nip * p.ncol;
    a.in_inner = a.out_inner = a.n_elem;
    a.m1 = c->m[0]; a.m2 = c->m[1]; a.m3 = c->m[2];
    a.mode = 1;
    a.sign = +1;
    a.scale = 1.0 / std::sqrt((double)nk);
    // the register pair transform of the mixed precisions reads psi as
    // complex FP32 (in the U region while it is free, or its own region)
    if (p.psi32) a.out32 = psi32;
    HIPCHK(kconv_launch(a, s));
  }
  if (timed) ws.timer.end("frag_t", s);
  const int nh = c->nh;
  const long long rows = p.nb == 1 ? p.ptot : p.pb;            // pair rows of the M / U regions
  const long long mplane = (long long)nh * rows * ld;
  // pair-transform tile of the LDS paths: ti interpolation points x tp
  // pairs, 64 KB of complex FP64 (nk * tp * ti <= 4096) or FP32 (<= 8192)
  const long long tile_cap = pair32_supported(prec, c->m[0], c->m[1], c->m[2]) ? 8192 : 4096;
  int ti = 32;
  while (ti > 1 && (long long)nk * ti > tile_cap) ti >>= 1;
  int tp = 1;   // power of two (the LDS transform needs tp * ti to be one)
  while (tp < 8 && (long long)nk * ti * tp * 2 <= tile_cap) tp *= 2;
  int ipair = 0;
  if (pair_lines_supported(prec, c->m[0], c->m[1], c->m[2])) {
    // the line transform: one value a thread an axis pass.  A tile whose LDS
    // would leave one workgroup a CU (the 10^3 mesh: 129 KB at 16 points) is
    // halved, the halves of each 16-point range run by neighbouring
    // workgroups (ipair; 86.6 against 91.1 ms a step at the 1000-k workload)
    ti = std::min(32, pair_lines_wmax(c->m[0], c->m[1], c->m[2]));
    tp = 1;
    if (ti >= 16 && pair_lines_lds(c->m[0], c->m[1], c->m[2], ti) > 80 * 1024) {
      ti /= 2;
      ipair = 1;
    }
  }
  const bool reg = pair_reg_supported(prec, c->m[0], c->m[1], c->m[2]);
  const long long nchunk = (ld + 63) / 64;
  // tables of the pair transform over pairs [pbeg, pbeg + pcnt) of every
  // fragment (unblocked: all pairs, output rows at the fragment's pair offset;
  // blocked: the block's pairs, output rows from 0)
  auto make_tables = [&](long long pbeg, long long pcnt) {
    PairTables t;
    std::vector<PairBlock> blocks;
    std::vector<long long> fpair(fr.size());
    std::vector<int> fp0(fr.size()), fnp(fr.size());
    std::vector<long long> ioff(fr.size() + 1, 0);
    for (size_t f = 0; f < fr.size(); ++f) {
      const long long np = p.nb == 1 ? (long long)p.nf[f] * p.nf[f] : pcnt;
      const long long b0 = p.nb == 1 ? 0 : pbeg;
      fp0[f] = (int)b0;
      fnp[f] = (int)np;
      fpair[f] = p.nb == 1 ? p.poff[f] : -b0;
      if (p.nb == 1 && tp == 1) {
        // single pairs of a whole fragment in windows of 8 rows p: for each
        // q, the pairs (p, q) of the window, so that consecutive blocks (run
        // together on one XCD) need 8 + a few orbitals of the point tile
        const int nfr = p.nf[f];
        for (int p0 = 0; p0 < nfr; p0 += 8)
          for (int q = 0; q < nfr; ++q)
            for (int pp = p0; pp < std::min(p0 + 8, nfr); ++pp) blocks.push_back(PairBlock{(int)f, pp * nfr + q, 1});
      } else {
        for (long long q0 = 0; q0 < np; q0 += tp)
          blocks.push_back(PairBlock{(int)f, (int)(b0 + q0), (int)std::min<long long>(tp, np - q0)});
      }
      ioff[f + 1] = ioff[f] + nchunk * np;
    }
    t.nblocks = (int)blocks.size();
    t.blocks = ws.arena.put(blocks.data(), blocks.size(), s);
    t.frag_pair = ws.arena.put(fpair.data(), fpair.size(), s);
    t.frag_p0 = ws.arena.put(fp0.data(), fp0.size(), s);
    t.frag_np = ws.arena.put(fnp.data(), fnp.size(), s);
    t.item_off = ws.arena.put(ioff.data(), ioff.size(), s);
    t.nitems = ioff.back();
    return t;
  };
  const int* d_nf = ws.arena.put(p.nf.data(), p.nf.size(), s);
  const int* d_col = ws.arena.put(p.col.data(), p.col.size(), s);
  // R^q_{I,pq} = N_k^{-1/2} sum_R exp(-iq.R) conj(psi_p) psi_q   (eq. (20)),
  // in the GEMM operand format of the precision, pair-major: row (pair) holds
  // the nh blocks of ld columns (class of q, I), so that the contraction over
  // (q, J) of every fragment reads one contiguous K range per row.  Only one
  // q of each class {q, -q} is kept: R^{-q}_{pq} = conj(R^q_{qp}).
  auto pair_transform = [&](const PairTables& t, char* out) {
    PairArgs a;
    memset(&a, 0, sizeof(a));
    a.psi = Tf;
    a.psi32 = p.psi32 ? psi32 : nullptr;
    a.out = out;
    a.blocks = t.blocks;
    a.frag_nf = d_nf;
    a.frag_col = d_col;
    a.frag_pair = t.frag_pair;
    a.frag_p0 = t.frag_p0;
    a.frag_np = t.frag_np;
    a.nblocks = t.nblocks;
    a.n_ip = nip;
    a.ncol = p.ncol;
    a.tp = tp;
    a.ti = ti;
    a.n_itiles = (int)((ld + ti - 1) / ti);
    a.ld = ld;
    a.q_stride = ld;                     // pair-major: [pair][class][I]
    a.p_stride = (long long)nh * ld;
    a.qslot = c->qmap.as<int>();
    a.plane = mplane;
    a.fmt = prec;
    a.m1 = c->m[0]; a.m2 = c->m[1]; a.m3 = c->m[2];
    a.scale = 1.0 / std::sqrt((double)nk);
    a.ipair = ipair;
    if (reg) {
      a.item_off = t.item_off;
      a.nfrag = (int)fr.size();
      a.nitems = t.nitems;
    }
    HIPCHK(pair_launch(a, s));
  };
  // U^q_{P,J} = sum_I R^q_{P,I} W^q_{IJ}   (eq. (19), first contraction)
  // With the factor (wfac, mixed precisions) the same product with W^T
  // replaced by sqrt(w_h) L^T: Y^q_{P,j} = sum_{a >= j} R^q_{P,a} L^q_{a,j}.
  const bool yform = prec != 0 && c->wfac;
  auto u_gemm = [&](const char* m, long long nrows, char* dst) {
    const void* wt = prec == 0 ? c->wt64.p : (prec == 1 ? c->wt32.p : (prec == 2 ? c->wt16.p : c->wt16s.p));
    std::vector<NtDesc> d(1);
    d[0] = mknt(m, (long long)nh * ld, wt, ld, dst, (long long)nh * ld, (int)nrows, nip, nip);
    d[0].ktri = yform ? 1 : 0;
    d[0].batch = nh;
    d[0].a_plane = mplane;
    d[0].b_plane = (long long)nh * nip * ld;
    d[0].c_plane = mplane;
    d[0].sA_bat = d[0].sC_bat = ld;
    d[0].sB_bat = (long long)nip * ld;
    d[0].epi = prec == 0 ? 0 : 3;
    d[0].npad = (int)ld;
    if (prec == 0) run_nt(ws.arena, prec, 0, d, s, 2);
    else run_big(ws.arena, prec, 0, d, 1, s, 2);
  };
  // (pq|rs) = sum_q sum_J U^q_{(pq),J} conj(R^q_{(sr),J})  (eq. (19), R^{-q}_{rs} = conj R^q_{sr}).
  // The term of -q is the conjugate of that of q with (pq) -> (qp) and
  // (sr) -> (rs) (R^{-q}_{pq} = conj R^q_{qp}, W^{-q} = conj W^q), so the
  // contraction runs over one q per class {q, -q} (weight 1/2 where q = -q,
  // folded into W):  G_f[(pq)][(sr)] = sum_{h, J} U^h_{(pq),J} conj(R^h_{(sr),J})
  // in FP64 (lower triangle; one grouped persistent launch over all
  // fragments, or one per block pair), then (pq|rs) = G[(pq)][(sr)] +
  // conj(G[(qp)][(rs)]) by the scatter.  FP64 path: FP64 sum over the
  // classes inside the kernel; mixed: one launch per group of classes (one
  // contiguous K range per row, FP32 sums inside), FP64 sum over the groups.
  const size_t sc = fmt_scalar(prec);
  const int ngroup = (nh + c->eri_qgroup - 1) / c->eri_qgroup;
  const int qgroup = (nh + ngroup - 1) / ngroup;       // balanced groups
  auto eri_desc = [&](const void* A, const void* B, cplx* C, long long ldc, int M, int N, int herm) {
    NtDesc g = mknt(A, (long long)nh * ld, B, (long long)nh * ld, C, ldc, M, N, nip);
    g.a_plane = g.b_plane = mplane;
    g.herm = herm;
    if (prec == 0) {
      g.nseg = nh;
      g.sA_seg = g.sB_seg = ld;
      g.epi = 0;
    } else {
      g.Kseg = (int)(qgroup * ld);
      g.nseg = (nh + qgroup - 1) / qgroup;
      g.Klast = (int)((nh - (long long)(g.nseg - 1) * qgroup) * ld);
      g.sA_seg = g.sB_seg = qgroup * ld;
      g.epi = 1;
    }
    return g;
  };
  // the GEMM launches alone, timed as "frag_eri_kernel" (one interval per launch)
  LaunchMark mark = nullptr;
  if (timed)
    mark = [&](bool on) {
      if (on) ws.timer.begin("frag_eri_kernel", s);
      else ws.timer.end("frag_eri_kernel", s);
    };
  auto eri_gemm = [&](std::vector<NtDesc>& d) {
    if (prec == 0) run_nt(ws.arena, prec, 2, d, s, 3, mark);
    else run_big(ws.arena, prec, 2, d, d[0].nseg, s, 3, mark);
  };
  if (p.nb == 1) {
    if (timed) ws.timer.begin("frag_pair", s);
    pair_transform(make_tables(0, 0), Mq);
    if (timed) ws.timer.end("frag_pair", s);
    if (timed) ws.timer.begin("frag_u", s);
    u_gemm(Mq, p.ptot, Uq);
    if (timed) ws.timer.end("frag_u", s);
    if (timed) ws.timer.begin("frag_eri", s);
    std::vector<NtDesc> d;
    for (size_t f = 0; f < fr.size(); ++f) {
      const int nf2 = p.nf[f] * p.nf[f];
      const size_t o = (size_t)p.poff[f] * nh * ld * sc;
      // G = U R^H, or Y Y^H with the factor
      d.push_back(eri_desc(Uq + o, (yform ? Uq : Mq) + o, acc + p.aoff[f], nf2, nf2, nf2, 2));
    }
    // largest fragments first so the persistent launch ends balanced
    std::stable_sort(d.begin(), d.end(), [](const NtDesc& a, const NtDesc& b) { return a.M > b.M; });
    eri_gemm(d);
  } else {
    // (pq)-blocked fragment (eqs. (19)-(20) over pair blocks): for row block
    // i, R^q_i and U^q_i = R^q_i W^q; for every column block j <= i, R^q_j
    // (recomputed into the second R region unless j == i) and the block
    // G[B_i][B_j] = U_i R_j^H (the lower tiles where j == i)
    const long long nf2 = (long long)p.nf[0] * p.nf[0];
    std::vector<PairTables> tabs(p.nb);
    for (int b = 0; b < p.nb; ++b) {
      const long long b0 = (long long)b * p.pb;
      tabs[b] = make_tables(b0, std::min<long long>(p.pb, nf2 - b0));
    }
    for (int i = 0; i < p.nb; ++i) {
      const long long i0 = (long long)i * p.pb, ni = std::min<long long>(p.pb, nf2 - i0);
      if (timed) ws.timer.begin("frag_pair", s);
      pair_transform(tabs[i], Mq);
      if (timed) ws.timer.end("frag_pair", s);
      if (timed) ws.timer.begin("frag_u", s);
      u_gemm(Mq, ni, Uq);
      if (timed) ws.timer.end("frag_u", s);
      for (int j = 0; j <= i; ++j) {
        const long long j0 = (long long)j * p.pb, nj = std::min<long long>(p.pb, nf2 - j0);
        // column operand: R_j, or with the factor Y_j (Y_i for j == i; else
        // Y_j = R_j L into the first R region, whose R_i is no longer read)
        const char* rj = yform ? Uq : Mq;
        if (j != i) {
          if (timed) ws.timer.begin("frag_pair", s);
          pair_transform(tabs[j], Mq2);
          if (timed) ws.timer.end("frag_pair", s);
          rj = Mq2;
          if (yform) {
            if (timed) ws.timer.begin("frag_u", s);
            u_gemm(Mq2, nj, Mq);
            if (timed) ws.timer.end("frag_u", s);
            rj = Mq;
          }
        }
        if (timed) ws.timer.begin("frag_eri", s);
        std::vector<NtDesc> d(1, eri_desc(Uq, rj, acc + i0 * nf2 + j0, nf2, (int)ni, (int)nj, j == i ? 2 : 0));
        eri_gemm(d);
        if (timed) ws.timer.end("frag_eri", s);
      }
    }
    if (timed) ws.timer.begin("frag_eri", s);
  }
  {
    std::vector<cplx*> outs(fr.size());
    for (size_t f = 0; f < fr.size(); ++f)
      outs[f] = (fr[f].flags & ISDF_FRAG_DEVICE) ? (cplx*)fr[f].eri : Est + p.eoff[f];
    HIPCHK(eri_scatter_batch_launch(acc, ws.arena.put(p.aoff.data(), p.aoff.size(), s),
                                    ws.arena.put(outs.data(), outs.size(), s), d_nf, (int)fr.size(), maxnf, s));
  }
  if (timed) ws.timer.end("frag_eri", s);
  for (size_t f = 0; f < fr.size(); ++f) {
    if (fr[f].flags & ISDF_FRAG_DEVICE) continue;
    const long long e4 = (long long)p.nf[f] * p.nf[f] * p.nf[f] * p.nf[f];
    HIPCHK(hipMemcpyAsync(fr[f].eri, Est + p.eoff[f], e4 * sizeof(cplx), hipMemcpyDeviceToHost, s));
  }
}

// Memory a synchronous fragment call may use: what is free on the device
// plus what the workspace already holds, less a margin.
size_t sync_cap(const Workspace& ws) {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return ws.mem.bytes;
  }
  const size_t avail = fr + ws.mem.bytes;
  const size_t margin = std::max<size_t>((size_t)1 << 28, avail / 16);
  return avail > margin ? avail - margin : 0;
}

// Run a list of fragments on ws within `cap` bytes of workspace: greedy
// sub-batches of consecutive fragments whose unblocked workspace fits, and a
// fragment that does not fit alone runs (pq)-blocked.  Sub-batches after the
// first wait for the previous one (the workspace is reused).
void enqueue_fragments(isdf_ctx c, Workspace& ws, int prec, const std::vector<FragIn>& fr, bool timed,
                       size_t cap) {
  // every fragment must fit (blocked if need be) before anything is enqueued
  std::vector<int> nbs(fr.size());
  for (size_t i = 0; i < fr.size(); ++i) {
    nbs[i] = blocks_for(c, fr[i], prec, cap);
    if (nbs[i] == 0)
      throw Fail{ISDF_E_NOMEM, "fragment " + std::to_string(i) + " (" + std::to_string(fr[i].nf) +
                                   " orbitals) does not fit the " + std::to_string(cap >> 20) +
                                   " MiB workspace even in " + std::to_string(MAX_PAIR_BLOCKS) + " pair blocks"};
  }
  size_t i = 0;
  while (i < fr.size()) {
    std::vector<FragIn> sub(1, fr[i]);
    const int nb = nbs[i];
    size_t j = i + 1;
    if (nb == 1)
      while (j < fr.size()) {
        sub.push_back(fr[j]);
        if (batch_bytes(c, sub, prec, 1) > cap) {
          sub.pop_back();
          break;
        }
        ++j;
      }
    enqueue_batch(c, ws, prec, sub, timed, nb);
    i = j;
  }
}

// Checks that every C[f] and eri[f] is device memory (callers that hand the
// pointers to kernels without staging).
void require_device(const void* const* C, void* const* eri, int n) {
  for (int f = 0; f < n; ++f) {
    hipPointerAttribute_t a1, a2;
    if (hipPointerGetAttributes(&a1, C[f]) != hipSuccess || hipPointerGetAttributes(&a2, eri[f]) != hipSuccess ||
        a1.type != hipMemoryTypeDevice || a2.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      throw Fail{ISDF_E_INVALID, "fragment " + std::to_string(f) + " needs device pointers for C and eri"};
    }
  }
}

// --------------------------------------------------------------------------
// serving thread
// --------------------------------------------------------------------------

void serve_loop(isdf_ctx c) {
  std::vector<Workspace*> inflight;
  while (true) {
    // retire finished batches
    for (size_t i = 0; i < inflight.size();) {
      Workspace* ws = inflight[i];
      hipError_t q = hipEventQuery(ws->done);
      if (q == hipErrorNotReady) { ++i; continue; }
      const double t = now_s();
      std::lock_guard<std::mutex> lk(c->mu);
      if (q == hipSuccess) ws->timer.collect(&c->totals);
      --c->inflight_n;
      for (uint64_t tk : ws->tickets) {
        auto it = c->reqs.find(tk);
        if (it == c->reqs.end()) continue;
        if (q == hipSuccess) {
          it->second.state = ISDF_REQ_DONE;
        } else {
          it->second.state = ISDF_REQ_FAILED;
          it->second.err = hipGetErrorString(q);
        }
        it->second.t_done = t;
        ++c->served;
      }
      ws->tickets.clear();
      c->ws_pool.push_back(ws);
      inflight.erase(inflight.begin() + i);
      c->cv.notify_all();
    }
    // admit a new batch
    Workspace* ws = nullptr;
    std::vector<FragIn> fr;
    std::vector<uint64_t> tks;
    int prec = 0;
    {
      std::unique_lock<std::mutex> lk(c->mu);
      if (c->stop && c->queue.empty() && inflight.empty()) break;
      // nothing is admitted while a synchronous call holds the context
      // (isdf_fit, isdf_coulomb_kernel, isdf_autotune, isdf_set_tiling)
      if (!c->exclusive && !c->ws_pool.empty() && !c->queue.empty()) {
        // a batch's fragments fit the per-batch budget unblocked together
        // (the sum of their single-fragment workspaces bounds the batch's);
        // a request that fits only (pq)-blocked runs alone
        long long used = 0;
        while (!c->queue.empty() && (int)fr.size() < c->max_batch) {
          uint64_t tk = c->queue.front();
          auto it = c->reqs.find(tk);
          if (it == c->reqs.end() || it->second.state != ISDF_REQ_QUEUED) {
            c->queue.pop_front();
            continue;
          }
          const isdf_request& r = it->second.req;
          if (!fr.empty() && r.prec != prec) break;
          const FragIn fi{r.n_f, r.C, r.eri, r.flags};
          const long long b = (long long)batch_bytes(c, std::vector<FragIn>(1, fi), r.prec, 1);
          if (!fr.empty() && used + b > serve_cap(c)) break;
          if (fr.empty()) prec = r.prec;
          used += b;
          fr.push_back(fi);
          tks.push_back(tk);
          it->second.state = ISDF_REQ_RUNNING;
          c->queue.pop_front();
          if (b > serve_cap(c)) break;          // blocked: alone in its batch
        }
        if (!fr.empty()) {
          ws = c->ws_pool.back();
          c->ws_pool.pop_back();
          ++c->inflight_n;                      // in flight from the moment its requests left the queue
        }
      } else if (inflight.empty()) {
        c->cv.wait_for(lk, std::chrono::microseconds(200));
        continue;
      }
    }
    if (ws) {
      try {
        enqueue_fragments(c, *ws, prec, fr, true, (size_t)serve_cap(c));
        HIPCHK(hipEventRecord(ws->done, ws->stream));
        ws->tickets = tks;
        inflight.push_back(ws);
        std::lock_guard<std::mutex> lk(c->mu);
        ++c->batches;
      } catch (const Fail& e) {
        (void)hipStreamSynchronize(ws->stream);
        std::lock_guard<std::mutex> lk(c->mu);
        --c->inflight_n;
        c->cv.notify_all();
        for (uint64_t tk : tks) {
          auto& r = c->reqs[tk];
          r.state = ISDF_REQ_FAILED;
          r.err = e.msg;
          r.t_done = now_s();
        }
        c->serve_err = e.msg;
        c->ws_pool.push_back(ws);
      }
    } else {
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
}

#ifndef ISDF_RHS_TILE_BYTES
#define ISDF_RHS_TILE_BYTES (1LL << 30)
#endif

// Tile of the right-hand side, T^k_I(r) for every k of rc grid points x ri
// interpolation points, within ISDF_RHS_TILE_BYTES (the environment variable
// of that name overrides it): every point and as many grid points as fit,
// else (fewer than 256 grid points would fit) 256 grid points and a balanced
// range of points, a multiple of 16 -- the pre-product reuses each X value
// over the tile's grid points, so the grid points are kept.
struct RhsTile { long long rc; int ri; };
RhsTile rhs_tile(long long ng, int nk, int nip) {
  long long budget = ISDF_RHS_TILE_BYTES;
  if (const char* v = std::getenv("ISDF_RHS_TILE_BYTES")) {
    const long long x = std::atoll(v);
    if (x > 0) budget = x;
  }
  const long long per_point = (long long)nk * (long long)sizeof(cplx);
  const long long rmin = std::min<long long>(ng, 256);
  const long long rc = budget / (per_point * nip);
  if (rc >= rmin) return {std::min(rc, ng), nip};
  long long ri = std::max<long long>(16, budget / (per_point * rmin) / 16 * 16);
  const long long nt = (nip + ri - 1) / ri;
  ri = std::min<long long>(nip, ((nip + nt - 1) / nt + 15) / 16 * 16);
  return {rmin, (int)ri};
}

// Sizes, reciprocal lattice, classes {q, -q}, the resident buffers (X, Pi,
// W and its operand copies, the factor's rank and permutation), the
// streams and events.  with_orbitals: also the orbitals and the fit's
// transient buffers (a context restored by isdf_load has neither).
void setup_context(isdf_ctx c, const double* lattice, const int32_t grid[3], const int32_t kmesh[3], int n_orb,
                   int n_ip, uint32_t flags, void* hip_stream, bool with_orbitals) {
  for (int d = 0; d < 3; ++d) { c->n[d] = grid[d]; c->m[d] = kmesh[d]; }
  c->nk = kmesh[0] * kmesh[1] * kmesh[2];
  c->ng = (long long)grid[0] * grid[1] * grid[2];
  c->norb = n_orb;
  c->nip = n_ip;
  c->flags = flags;
  c->stream = (hipStream_t)hip_stream;
  c->has_orbitals = with_orbitals;
  HIPCHK(hipGetDevice(&c->device));
  memcpy(c->lattice, lattice, sizeof(c->lattice));
  // reciprocal rows b_i: 2 pi (A^-1)^T
  const double* A = lattice;
  const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                     A[2] * (A[3] * A[7] - A[4] * A[6]);
  if (!(std::fabs(det) > 1e-12)) throw Fail{ISDF_E_INVALID, "singular lattice"};
  c->volume = std::fabs(det);
  double inv[9];
  inv[0] = (A[4] * A[8] - A[5] * A[7]) / det;
  inv[1] = (A[2] * A[7] - A[1] * A[8]) / det;
  inv[2] = (A[1] * A[5] - A[2] * A[4]) / det;
  inv[3] = (A[5] * A[6] - A[3] * A[8]) / det;
  inv[4] = (A[0] * A[8] - A[2] * A[6]) / det;
  inv[5] = (A[2] * A[3] - A[0] * A[5]) / det;
  inv[6] = (A[3] * A[7] - A[4] * A[6]) / det;
  inv[7] = (A[1] * A[6] - A[0] * A[7]) / det;
  inv[8] = (A[0] * A[4] - A[1] * A[3]) / det;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c->recip[3 * i + j] = 2.0 * M_PI * inv[3 * j + i];
  const int nk = c->nk;
  const long long ng = c->ng;
  const size_t e = sizeof(cplx);
  c->qslot_h.assign(nk, -1);
  for (int q = 0; q < nk; ++q) {
    const int j1 = q / (c->m[1] * c->m[2]), j2 = (q / c->m[2]) % c->m[1], j3 = q % c->m[2];
    const int mq = (((c->m[0] - j1) % c->m[0]) * c->m[1] + (c->m[1] - j2) % c->m[1]) * c->m[2] +
                   (c->m[2] - j3) % c->m[2];
    if (mq < q) continue;
    c->qslot_h[q] = (int)c->hq_h.size();
    c->hq_h.push_back(q);
    c->hself_h.push_back(mq == q ? 1 : 0);
  }
  c->nh = (int)c->hq_h.size();
  {
    const RhsTile t = rhs_tile(ng, nk, n_ip);
    c->rc = t.rc;
    c->ri = t.ri;
  }
  if (with_orbitals) c->phi.alloc((size_t)nk * n_orb * ng * e);
  c->ip.alloc(sizeof(int) * n_ip);
  // + RHS_X_PAD elements: rhs_t_launch reads whole blocks of points
  c->xt.alloc(((size_t)nk * n_orb * n_ip + RHS_X_PAD) * e);
  const int nh = c->nh;
  const size_t m2 = (size_t)nh * n_ip * n_ip * e;   // one matrix per class {q, -q}
  c->pi.alloc(m2);
  c->w.alloc(m2);
  // row pitches of the split operands: multiples of 16 elements, so that in
  // the bf16 hi/lo format every 16-k step of a row is one aligned 128-byte line
  c->ld_ip = (n_ip + 15) / 16 * 16;
  c->eri_qgroup = c->eri_qgroup0 = initial_qgroup(c->ld_ip);
  c->wt64.alloc((size_t)nh * n_ip * c->ld_ip * e);
  c->wt32.alloc((size_t)nh * n_ip * c->ld_ip * 8);
  c->wt16.alloc((size_t)nh * n_ip * c->ld_ip * 8);
  c->wt16s.alloc((size_t)nh * n_ip * c->ld_ip * 4);
  c->perm.alloc(sizeof(int) * nh * n_ip);
  c->rank.alloc(sizeof(int) * nh);
  c->flag.alloc(sizeof(int));
  c->dmax.alloc(sizeof(double) * nh);
  c->cflag.alloc(sizeof(int) * nh);
  if (with_orbitals) {
    // classes per q batch of eta: all of them when that fits in 60 % of the
    // memory left after the resident and the other transient buffers (the
    // rest is for fragment workspaces), else the largest batch that fits in
    // 85 % of it -- a q-batched kernel hands the transient buffers back to
    // the fragment workspaces when it ends.  ISDF_Q_BATCH(n) caps the batch.
    const size_t per_class = (size_t)n_ip * ng * e;
    const size_t transient = 3 * m2 + (size_t)nk * n_ip * n_ip * e +
                             (size_t)nh * ((size_t)n_ip * 64 + 4096) * e + 2 * (size_t)nk * c->ri * c->rc * e;
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    const double avail = fr > transient ? (double)(fr - transient) : 0.0;
    long long qb = (long long)(0.6 * avail / (double)per_class);
    if (qb < nh) qb = (long long)(0.85 * avail / (double)per_class);
    const int cap = (int)((flags >> 16) & 0xFFFFu);
    if (cap > 0) qb = std::min<long long>(qb, cap);
    if (qb < 1) throw Fail{ISDF_E_NOMEM, "no room for the eta of one q class"};
    c->qb = (int)std::min<long long>(qb, nh);
    ensure_fit_buffers(c);
  }
  c->qmap.alloc(sizeof(int) * (nk + 2 * c->nh));
  {
    std::vector<int> qm(c->qslot_h);
    qm.insert(qm.end(), c->hq_h.begin(), c->hq_h.end());
    qm.insert(qm.end(), c->hself_h.begin(), c->hself_h.end());
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(c->qmap.p, qm.data(), sizeof(int) * qm.size(), hipMemcpyHostToDevice));
  }
  c->sync_ws.stream = c->stream;
  // this device's copy of the static workspace array
  c->scratch = scratch_ptr(c->device);
  HIPCHK(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&c->aux2, hipStreamNonBlocking));
  for (int b = 0; b < 2; ++b) {
    HIPCHK(hipEventCreateWithFlags(&c->ev_rt[b], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_kc[b], hipEventDisableTiming));
  }
  HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c->ev_pinv, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c->sync_ws.done, hipEventDisableTiming));
}

const char* check_sizes(const int32_t grid[3], const int32_t kmesh[3], int32_t n_orb, int32_t n_ip) {
  for (int d = 0; d < 3; ++d) {
    if (!good_grid(grid[d])) return "grid size must be 2..64 with factors 2,3,5,7";
    if (kmesh[d] < 1 || kmesh[d] > 16) return "k mesh must be 1..16 per axis";
  }
  if (n_orb < 1 || n_orb > 256 || n_ip < 1 || n_ip > 2048) return "n_orb must be 1..256 and n_ip 1..2048";
  return nullptr;
}

// Interpolation points: in range and distinct.
void check_ips(const std::vector<int32_t>& iph, long long ng) {
  std::vector<int32_t> srt(iph);
  std::sort(srt.begin(), srt.end());
  if (srt.front() < 0 || srt.back() >= ng) throw Fail{ISDF_E_INVALID, "interpolation point index out of range"};
  for (size_t i = 1; i < srt.size(); ++i)
    if (srt[i] == srt[i - 1]) throw Fail{ISDF_E_INVALID, "duplicate interpolation point"};
}

// --------------------------------------------------------------------------
// checkpoint files (isdf_save / isdf_load)
// --------------------------------------------------------------------------
// Little-endian.  Header (CkHeader), then the payload:
//   int32 ip_index[n_ip]; int32 rank[nh];
//   c128 X[N_k][n_orb][n_ip] (the context's layout);
//   c128 Pi[nh][n_ip][n_ip]; c128 W[nh][n_ip][n_ip] (one q per class {q, -q},
//   class h = the h-th q of the mesh whose -q is not smaller)
// checksum = FNV-1a 64 over the payload bytes.
struct CkHeader {
  char magic[8];            // "ISDFCKP1"
  uint32_t version;         // 1
  uint32_t header_bytes;    // sizeof(CkHeader)
  int32_t grid[3], kmesh[3], n_orb, n_ip, nh;
  uint32_t flags;           // isdf_create flags of the saved context
  double lattice[9];
  uint64_t payload_bytes;
  uint64_t checksum;
};
static_assert(sizeof(CkHeader) == 8 + 4 + 4 + 4 * 9 + 4 + 72 + 8 + 8, "checkpoint header layout");
const char kCkMagic[8] = {'I', 'S', 'D', 'F', 'C', 'K', 'P', '1'};

uint64_t fnv1a(uint64_t h, const unsigned char* p, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}
constexpr uint64_t kFnvInit = 1469598103934665603ull;

int classes_of(const int32_t kmesh[3]) {
  long long nself = 1;
  for (int d = 0; d < 3; ++d) nself *= (kmesh[d] % 2 == 0) ? 2 : 1;
  return (int)(((long long)kmesh[0] * kmesh[1] * kmesh[2] + nself) / 2);
}

uint64_t ck_payload_bytes(const CkHeader& h) {
  const uint64_t nk = (uint64_t)h.kmesh[0] * h.kmesh[1] * h.kmesh[2];
  return 4ull * h.n_ip + 4ull * h.nh + 16ull * nk * h.n_orb * h.n_ip + 2ull * 16 * h.nh * h.n_ip * h.n_ip;
}

}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

const char* isdf_version(void) { return kVersion; }

int64_t isdf_storage_model_bytes(int64_t n_k, int64_t n_ip, int64_t n_ao) {
  return (n_k * n_ip * n_ip + n_k * n_ip * n_ao) * 16;
}

int64_t isdf_plan_bytes(const int32_t grid[3], const int32_t kmesh[3], int32_t n_orb, int32_t n_ip) {
  if (!grid || !kmesh) return -1;
  const long long ng = (long long)grid[0] * grid[1] * grid[2];
  const long long nk = (long long)kmesh[0] * kmesh[1] * kmesh[2];
  // classes {q, -q}: (N_k + number of q = -q) / 2, q = -q where every axis is 0 or m/2
  long long nself = 1;
  for (int d = 0; d < 3; ++d) nself *= (kmesh[d] % 2 == 0) ? 2 : 1;
  const long long nh = (nk + nself) / 2;
  const long long e = sizeof(cplx);
  const long long ld = (n_ip + 15) / 16 * 16;
  long long b = 0;
  b += nk * n_orb * ng * e;              // orbitals
  b += nk * n_orb * n_ip * e;            // X
  b += nk * (long long)n_ip * n_ip * e;  // T^k of the metric, then V
  b += 5 * nh * (long long)n_ip * n_ip * e;  // Pi, L, W, two work buffers (per class)
  b += nh * ((long long)n_ip * 64 + 4096) * e;  // L^{-1} scratch
  b += nh * (long long)n_ip * ld * (16 + 8 + 8 + 4);  // W^T in the four operand formats
  b += nh * (long long)n_ip * ng * e;    // eta of every class (q batches need less)
  {
    const RhsTile t = rhs_tile(ng, (int)nk, n_ip);
    b += 2 * nk * (long long)t.ri * t.rc * e;  // two RHS tiles
  }
  b += n_ip * 4 + 2 * nh * (long long)n_ip * 4;
  return b;
}


isdf_status isdf_create(isdf_ctx* out, const double* lattice, const int32_t grid[3],
                        const int32_t kmesh[3], int32_t n_orb, const void* orbitals,
                        const int32_t* ip_index, int32_t n_ip, uint32_t flags, void* hip_stream) {
  t_create_err.clear();
  if (!out) { t_create_err = "null output handle"; return ISDF_E_INVALID; }
  *out = nullptr;
  if (!lattice || !grid || !kmesh || !orbitals || !ip_index) {
    t_create_err = "null argument";
    return ISDF_E_INVALID;
  }
  if (const char* m = check_sizes(grid, kmesh, n_orb, n_ip)) {
    t_create_err = m;
    return ISDF_E_INVALID;
  }
  isdf_ctx c = new (std::nothrow) isdf_ctx_s();
  if (!c) return ISDF_E_NOMEM;
  isdf_status st = guarded(c, [&] {
    // validate interpolation points (host copy if needed)
    std::vector<int32_t> iph(n_ip);
    if (flags & ISDF_INPUT_DEVICE) {
      HIPCHK(hipMemcpy(iph.data(), ip_index, sizeof(int32_t) * n_ip, hipMemcpyDeviceToHost));
    } else {
      memcpy(iph.data(), ip_index, sizeof(int32_t) * n_ip);
    }
    check_ips(iph, (long long)grid[0] * grid[1] * grid[2]);
    setup_context(c, lattice, grid, kmesh, n_orb, n_ip, flags, hip_stream, true);
    const hipMemcpyKind kind = (flags & ISDF_INPUT_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(hipMemcpyAsync(c->phi.p, orbitals, (size_t)c->nk * n_orb * c->ng * sizeof(cplx), kind, c->stream));
    HIPCHK(hipMemcpyAsync(c->ip.p, iph.data(), sizeof(int) * n_ip, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
  if (st != ISDF_OK) {
    t_create_err = c->err;
    delete c;
    return st;
  }
  *out = c;
  return ISDF_OK;
}

isdf_status isdf_select_points(const int32_t grid[3], const int32_t kmesh[3], int32_t n_orb, const void* orbitals,
                               int32_t n_ip, int32_t* ip_out, double* residual_out, uint32_t flags,
                               void* hip_stream) {
  t_create_err.clear();
  if (!grid || !kmesh || !orbitals || !ip_out) {
    t_create_err = "null argument";
    return ISDF_E_INVALID;
  }
  if (const char* m = check_sizes(grid, kmesh, n_orb, n_ip)) {
    t_create_err = m;
    return ISDF_E_INVALID;
  }
  const long long ng = (long long)grid[0] * grid[1] * grid[2];
  const long long nrows = (long long)kmesh[0] * kmesh[1] * kmesh[2] * n_orb;
  if (n_ip > ng) {
    t_create_err = "n_ip exceeds the number of grid points";
    return ISDF_E_INVALID;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    if (flags & ISDF_INPUT_DEVICE) {
      hipPointerAttribute_t at;
      if (hipPointerGetAttributes(&at, orbitals) != hipSuccess || at.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        throw Fail{ISDF_E_INVALID, "ISDF_INPUT_DEVICE orbitals are not device memory"};
      }
    }
    const SelPlan pl = sel_plan(nrows, ng);
    DevBuf phi, part, lf, d, bv, bi, piv, dmax;
    const cplx* ph = (const cplx*)orbitals;
    if (!(flags & ISDF_INPUT_DEVICE)) {
      phi.alloc(sizeof(cplx) * nrows * ng);
      HIPCHK(hipMemcpyAsync(phi.p, orbitals, sizeof(cplx) * nrows * ng, hipMemcpyHostToDevice, s));
      ph = phi.as<cplx>();
    }
    part.alloc(sizeof(cplx) * pl.nslice * ng);
    lf.alloc(sizeof(double) * n_ip * ng);
    d.alloc(sizeof(double) * ng);
    bv.alloc(sizeof(double) * pl.xblocks);
    bi.alloc(sizeof(long long) * pl.xblocks);
    piv.alloc(sizeof(int) * n_ip);
    dmax.alloc(sizeof(double) * n_ip);
    HIPCHK(sel_start_launch(pl, ph, nrows, ng, part.as<cplx>(), d.as<double>(), bv.as<double>(),
                            bi.as<long long>(), piv.as<int>(), dmax.as<double>(), s));
    for (int i = 0; i < n_ip; ++i)
      HIPCHK(sel_step_launch(pl, ph, nrows, ng, part.as<cplx>(), lf.as<double>(), d.as<double>(), bv.as<double>(),
                             bi.as<long long>(), piv.as<int>(), dmax.as<double>(), i, i + 1 < n_ip, s));
    std::vector<int32_t> ph_piv(n_ip);
    std::vector<double> ph_dmax(n_ip);
    HIPCHK(hipMemcpyAsync(ph_piv.data(), piv.p, sizeof(int) * n_ip, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(ph_dmax.data(), dmax.p, sizeof(double) * n_ip, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // a step whose largest residual is not positive (the products span fewer
    // columns, or the orbitals hold non-finite values) ends the selection
    int good = 0;
    while (good < n_ip && ph_dmax[good] > 0.0 && ph_piv[good] >= 0 && ph_piv[good] < ng) ++good;
    for (int i = 0; i < n_ip; ++i) {
      ip_out[i] = i < good ? ph_piv[i] : -1;
      if (residual_out) residual_out[i] = i < good ? ph_dmax[i] : 0.0;
    }
    if (good < n_ip)
      throw Fail{ISDF_E_NUMERIC, "the pair products span only " + std::to_string(good) +
                                     " grid columns (largest residual not positive at step " +
                                     std::to_string(good) + ")"};
  } catch (const Fail& e) {
    t_create_err = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    t_create_err = "host allocation failed";
    return ISDF_E_NOMEM;
  } catch (...) {
    t_create_err = "unexpected exception";
    return ISDF_E_INVALID;
  }
  return ISDF_OK;
}

isdf_status isdf_fit(isdf_ctx ctx, isdf_precision prec) {
  return guarded(ctx, [&] {
    if (prec < ISDF_FP64 || prec > ISDF_MIXED_BF16) throw Fail{ISDF_E_INVALID, "bad precision"};
    if (!ctx->has_orbitals) throw Fail{ISDF_E_STATE, "context restored from a checkpoint has no orbitals to fit"};
    Exclusive ex(ctx, true);
    do_fit(ctx, prec);
  });
}


isdf_status isdf_coulomb_kernel(isdf_ctx ctx, isdf_precision prec) {
  return guarded(ctx, [&] {
    if (prec < ISDF_FP64 || prec > ISDF_MIXED_BF16) throw Fail{ISDF_E_INVALID, "bad precision"};
    if (!ctx->fitted || !ctx->kernel_pending)
      throw Fail{ISDF_E_STATE, "isdf_fit must run before isdf_coulomb_kernel"};
    Exclusive ex(ctx, true);
    do_kernel(ctx, prec);
  });
}

static isdf_status get_mat(isdf_ctx ctx, const DevBuf& b, long long off, size_t bytes, void* out) {
  return guarded(ctx, [&] {
    HIPCHK(hipMemcpyAsync(out, b.as<char>() + off, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

// Index of -q on the k mesh, and for a q of no stored class its partner:
// the stored class slot of q or of -q, and whether the value is conjugated.
static int minus_q_index(isdf_ctx c, int q) {
  const int j1 = q / (c->m[1] * c->m[2]), j2 = (q / c->m[2]) % c->m[1], j3 = q % c->m[2];
  return (((c->m[0] - j1) % c->m[0]) * c->m[1] + (c->m[1] - j2) % c->m[1]) * c->m[2] + (c->m[2] - j3) % c->m[2];
}
static int class_slot(isdf_ctx c, int q, bool* conj) {
  const int h = c->qslot_h[q];
  *conj = h < 0;
  return h >= 0 ? h : c->qslot_h[minus_q_index(c, q)];
}

// Copy slot h of a [class][n][n] matrix set to host, conjugated for -q.
static isdf_status get_class_mat(isdf_ctx ctx, const DevBuf& b, int q, void* out) {
  bool cj;
  const int h = class_slot(ctx, q, &cj);
  const size_t bytes = (size_t)ctx->nip * ctx->nip * sizeof(cplx);
  isdf_status st = get_mat(ctx, b, (long long)h * bytes, bytes, out);
  if (st == ISDF_OK && cj) {
    cplx* o = (cplx*)out;
    for (size_t i = 0; i < (size_t)ctx->nip * ctx->nip; ++i) o[i].y = -o[i].y;
  }
  return st;
}

isdf_status isdf_get_metric(isdf_ctx ctx, int32_t q, void* out) {
  if (!ctx) return ISDF_E_INVALID;
  if (!ctx->fitted) return fail(ctx, ISDF_E_STATE, "metric not computed");
  if (q < 0 || q >= ctx->nk || !out) return fail(ctx, ISDF_E_INVALID, "bad q");
  return get_class_mat(ctx, ctx->pi, q, out);              // Pi^{-q} = conj Pi^q
}

isdf_status isdf_get_kernel(isdf_ctx ctx, int32_t q, void* out) {
  if (!ctx) return ISDF_E_INVALID;
  if (!ctx->kernel_ready) return fail(ctx, ISDF_E_STATE, "Coulomb kernel not computed");
  if (q < 0 || q >= ctx->nk || !out) return fail(ctx, ISDF_E_INVALID, "bad q");
  return get_class_mat(ctx, ctx->w, q, out);               // W^{-q} = conj W^q
}

isdf_status isdf_get_ivs(isdf_ctx ctx, int32_t k, void* out) {
  if (!ctx) return ISDF_E_INVALID;
  if (!ctx->fitted) return fail(ctx, ISDF_E_STATE, "X not computed");
  if (k < 0 || k >= ctx->nk || !out) return fail(ctx, ISDF_E_INVALID, "bad k");
  // device layout Xt[k][mu][I]; return [I][mu]
  std::vector<cplx> t((size_t)ctx->norb * ctx->nip);
  const size_t b = t.size() * sizeof(cplx);
  isdf_status st = get_mat(ctx, ctx->xt, (long long)k * b, b, t.data());
  if (st != ISDF_OK) return st;
  cplx* o = (cplx*)out;
  for (int mu = 0; mu < ctx->norb; ++mu)
    for (int I = 0; I < ctx->nip; ++I) o[(size_t)I * ctx->norb + mu] = t[(size_t)mu * ctx->nip + I];
  return ISDF_OK;
}

isdf_status isdf_get_rhs(isdf_ctx ctx, int32_t q, void* out) {
  if (!ctx) return ISDF_E_INVALID;
  if (!ctx->eta_valid)
    return fail(ctx, ISDF_E_STATE,
                "eta not available (fit first; consumed by the kernel; formed inside the kernel when q-batched)");
  if (q < 0 || q >= ctx->nk || !out) return fail(ctx, ISDF_E_INVALID, "bad q");
  const size_t n = (size_t)ctx->nip * ctx->ng;
  bool cj;                                                   // eta^{-q} = conj eta^q
  const int hs = class_slot(ctx, q, &cj);
  return guarded(ctx, [&] {
    cplx* o = (cplx*)out;
    HIPCHK(hipMemcpyAsync(o, ctx->eta.as<cplx>() + (long long)hs * n, n * sizeof(cplx), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (cj)
      for (size_t i = 0; i < n; ++i) o[i].y = -o[i].y;
  });
}

isdf_status isdf_get_eta_tilde(isdf_ctx ctx, int32_t q, void* out) {
  if (!ctx) return ISDF_E_INVALID;
  if (!ctx->kernel_ready) return fail(ctx, ISDF_E_STATE, "eta~ not computed (isdf_coulomb_kernel first)");
  if (!ctx->etat_valid) return fail(ctx, ISDF_E_STATE, "eta~ is not kept when the kernel runs in q batches");
  if (q < 0 || q >= ctx->nk || !out) return fail(ctx, ISDF_E_INVALID, "bad q");
  const long long nip = ctx->nip, ng = ctx->ng;
  // a q of no stored class: eta~^q(G) = conj(eta~^{-q}(G')) with G' the
  // index of -(G + q) - (-q) (per axis -s, or 1 - s where q sits on the
  // zone boundary of an even mesh), which the symmetric kernel weighs alike
  bool cj;
  const int hs = class_slot(ctx, q, &cj);
  const size_t b = (size_t)nip * ng * sizeof(cplx);
  isdf_status st = get_mat(ctx, ctx->eta, (long long)hs * b, b, out);
  if (st != ISDF_OK || !cj) return st;
  const int j[3] = {q / (ctx->m[1] * ctx->m[2]), (q / ctx->m[2]) % ctx->m[1], q % ctx->m[2]};
  int dl[3];
  for (int d = 0; d < 3; ++d) dl[d] = (ctx->m[d] % 2 == 0 && 2 * j[d] == ctx->m[d]) ? 1 : 0;
  cplx* o = (cplx*)out;
  std::vector<cplx> row(ng);
  for (long long i = 0; i < nip; ++i) {
    cplx* r = o + i * ng;
    for (long long g = 0; g < ng; ++g) {
      const int s1 = (int)(g / ((long long)ctx->n[1] * ctx->n[2])), s2 = (int)((g / ctx->n[2]) % ctx->n[1]),
                s3 = (int)(g % ctx->n[2]);
      const int t1 = ((dl[0] - s1) % ctx->n[0] + ctx->n[0]) % ctx->n[0];
      const int t2 = ((dl[1] - s2) % ctx->n[1] + ctx->n[1]) % ctx->n[1];
      const int t3 = ((dl[2] - s3) % ctx->n[2] + ctx->n[2]) % ctx->n[2];
      const cplx v = r[((long long)t1 * ctx->n[1] + t2) * ctx->n[2] + t3];
      row[g] = cmk(v.x, -v.y);
    }
    memcpy(r, row.data(), ng * sizeof(cplx));
  }
  return ISDF_OK;
}

isdf_status isdf_fragment_eri(isdf_ctx ctx, isdf_precision prec, int32_t n_frag, const int32_t* n_f,
                              const void* const* C, void* const* eri, uint32_t flags) {
  return guarded(ctx, [&] {
    if (n_frag < 1 || !n_f || !C || !eri) throw Fail{ISDF_E_INVALID, "bad fragment arguments"};
    if (prec < ISDF_FP64 || prec > ISDF_MIXED_BF16) throw Fail{ISDF_E_INVALID, "bad precision"};
    std::vector<FragIn> fr;
    for (int f = 0; f < n_frag; ++f) {
      if (n_f[f] < 1 || n_f[f] > ctx->nk * ctx->norb || !C[f] || !eri[f])
        throw Fail{ISDF_E_INVALID, "bad fragment " + std::to_string(f)};
      fr.push_back(FragIn{n_f[f], C[f], eri[f], flags});
    }
    const int forced = (int)((flags >> 8) & 0xFFu);
    if (forced > 1) {
      for (const FragIn& f : fr)
        enqueue_batch(ctx, ctx->sync_ws, prec, std::vector<FragIn>(1, f), true,
                      (int)std::min<long long>(forced, (long long)f.nf * f.nf));
    } else {
      enqueue_fragments(ctx, ctx->sync_ws, prec, fr, true, sync_cap(ctx->sync_ws));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->sync_ws.timer.collect(&ctx->totals);
    for (auto& kv : ctx->sync_ws.timer.ms) ctx->timer.ms[kv.first] = kv.second;
  });
}

isdf_status isdf_fragment_eri_static(isdf_ctx ctx, isdf_precision prec, int32_t n_frag, const int32_t* n_f,
                                     const void* const* C, void* const* eri, uint32_t flags) {
  return guarded(ctx, [&] {
    if (n_frag < 1 || !n_f || !C || !eri) throw Fail{ISDF_E_INVALID, "bad fragment arguments"};
    if (prec < ISDF_FP64 || prec > ISDF_MIXED_BF16) throw Fail{ISDF_E_INVALID, "bad precision"};
    if (!(flags & ISDF_FRAG_DEVICE)) throw Fail{ISDF_E_INVALID, "the static variant takes device pointers only"};
    if (!ctx->kernel_ready) throw Fail{ISDF_E_STATE, "isdf_coulomb_kernel must run before fragment ERIs"};
    if (!ctx->scratch) throw Fail{ISDF_E_STATE, "static workspace not set up"};
    std::vector<FragIn> fr;
    for (int f = 0; f < n_frag; ++f) {
      if (n_f[f] < 1 || n_f[f] > ctx->nk * ctx->norb || !C[f] || !eri[f])
        throw Fail{ISDF_E_INVALID, "bad fragment " + std::to_string(f)};
      fr.push_back(FragIn{n_f[f], C[f], eri[f], ISDF_FRAG_DEVICE});
    }
    require_device(C, eri, n_frag);
    Workspace& ws = ctx->static_ws;
    if (ws.mem.p != (char*)ctx->scratch + STATIC_DESC_BYTES) {
      ws.stream = ctx->stream;
      ws.arena.attach(ctx->scratch, STATIC_DESC_BYTES);
      ws.mem.attach((char*)ctx->scratch + STATIC_DESC_BYTES, STATIC_SCRATCH_BYTES - STATIC_DESC_BYTES);
    }
    // sub-batches and (pq)-blocking within the array; a fragment that does
    // not fit even in the largest blocking is refused before any launch
    enqueue_fragments(ctx, ws, prec, fr, false, STATIC_SCRATCH_BYTES - STATIC_DESC_BYTES);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

struct isdf_graph_s {
  isdf_ctx ctx = nullptr;
  Workspace ws;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t after = nullptr;     // work queued on the context's stream before a replay
  ~isdf_graph_s() {
    if (ws.stream) (void)hipStreamSynchronize(ws.stream);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (after) (void)hipEventDestroy(after);
  }
};

isdf_status isdf_graph_create(isdf_ctx ctx, isdf_precision prec, int32_t n_frag, const int32_t* n_f,
                              const void* const* C, void* const* eri, isdf_graph* out) {
  return guarded(ctx, [&] {
    if (!out || n_frag < 1 || !n_f || !C || !eri) throw Fail{ISDF_E_INVALID, "bad graph arguments"};
    *out = nullptr;
    if (prec < ISDF_FP64 || prec > ISDF_MIXED_BF16) throw Fail{ISDF_E_INVALID, "bad precision"};
    if (!ctx->kernel_ready) throw Fail{ISDF_E_STATE, "isdf_coulomb_kernel must run before fragment ERIs"};
    std::vector<FragIn> fr;
    for (int f = 0; f < n_frag; ++f) {
      if (n_f[f] < 1 || n_f[f] > ctx->nk * ctx->norb || !C[f] || !eri[f])
        throw Fail{ISDF_E_INVALID, "bad fragment " + std::to_string(f)};
      fr.push_back(FragIn{n_f[f], C[f], eri[f], ISDF_FRAG_DEVICE});
    }
    require_device(C, eri, n_frag);
    std::unique_ptr<isdf_graph_s> g(new isdf_graph_s());
    g->ctx = ctx;
    HIPCHK(hipStreamCreateWithFlags(&g->ws.stream, hipStreamNonBlocking));
    g->ws.own_stream = true;
    HIPCHK(hipEventCreateWithFlags(&g->after, hipEventDisableTiming));
    HIPCHK(hipEventRecord(g->after, ctx->stream));
    HIPCHK(hipStreamWaitEvent(g->ws.stream, g->after, 0));
    // eager pass: sizes the workspace and descriptor arena (no allocation may
    // happen under capture) and runs every launch once
    enqueue_batch(ctx, g->ws, prec, fr, false);
    HIPCHK(hipStreamSynchronize(g->ws.stream));
    HIPCHK(hipStreamBeginCapture(g->ws.stream, hipStreamCaptureModeThreadLocal));
    try {
      enqueue_batch(ctx, g->ws, prec, fr, false, 1, true);
    } catch (...) {
      hipGraph_t part = nullptr;
      (void)hipStreamEndCapture(g->ws.stream, &part);
      if (part) (void)hipGraphDestroy(part);
      throw;
    }
    HIPCHK(hipStreamEndCapture(g->ws.stream, &g->graph));
    HIPCHK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    *out = g.release();
  });
}

isdf_status isdf_graph_launch(isdf_graph g) {
  if (!g) return ISDF_E_INVALID;
  return guarded(g->ctx, [&] {
    if (!g->ctx->kernel_ready) throw Fail{ISDF_E_STATE, "isdf_coulomb_kernel must run before fragment ERIs"};
    HIPCHK(hipEventRecord(g->after, g->ctx->stream));
    HIPCHK(hipStreamWaitEvent(g->ws.stream, g->after, 0));
    HIPCHK(hipGraphLaunch(g->exec, g->ws.stream));
    HIPCHK(hipStreamSynchronize(g->ws.stream));
  });
}

isdf_status isdf_graph_destroy(isdf_graph g) {
  if (!g) return ISDF_E_INVALID;
  delete g;
  return ISDF_OK;
}

isdf_status isdf_set_tiling(isdf_ctx ctx, int32_t eri_qgroup, int32_t wg_per_cu) {
  return guarded(ctx, [&] {
    if (eri_qgroup < 1 || wg_per_cu < 0 || wg_per_cu > 8) throw Fail{ISDF_E_INVALID, "bad tiling"};
    Exclusive ex(ctx, false);
    ctx->eri_qgroup = eri_qgroup;
    ctx->frag_wg_per_cu = wg_per_cu;
  });
}

isdf_status isdf_autotune(isdf_ctx ctx, isdf_precision prec, int32_t n_frag, const int32_t* n_f,
                          const void* const* C, void* const* eri, isdf_tune_report* report) {
  return guarded(ctx, [&] {
    if (n_frag < 1 || !n_f || !C || !eri) throw Fail{ISDF_E_INVALID, "bad fragment arguments"};
    if (prec < ISDF_FP64 || prec > ISDF_MIXED_BF16) throw Fail{ISDF_E_INVALID, "bad precision"};
    if (!ctx->kernel_ready) throw Fail{ISDF_E_STATE, "isdf_coulomb_kernel must run before fragment ERIs"};
    std::vector<FragIn> fr;
    for (int f = 0; f < n_frag; ++f) {
      if (n_f[f] < 1 || n_f[f] > ctx->nk * ctx->norb || !C[f] || !eri[f])
        throw Fail{ISDF_E_INVALID, "bad fragment " + std::to_string(f)};
      fr.push_back(FragIn{n_f[f], C[f], eri[f], ISDF_FRAG_DEVICE});
    }
    // the candidates run on device pointers without staging
    require_device(C, eri, n_frag);
    Exclusive ex(ctx, false);
    const int nh = ctx->nh;
    // classes per launch for one, two and three launches over the classes,
    // and the initial tiling (balanced groups of at most eri_qgroup0)
    const int g0 = ctx->eri_qgroup0, nl0 = (nh + g0 - 1) / g0;
    const int def_g = (nh + nl0 - 1) / nl0;
    std::vector<int> groups = {def_g};
    for (int nl = 1; nl <= 3 && nl <= nh; ++nl) groups.push_back((nh + nl - 1) / nl);
    std::sort(groups.begin(), groups.end());
    groups.erase(std::unique(groups.begin(), groups.end()), groups.end());
    const int wgs[] = {1, 2, 4, 8};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int old_g = ctx->eri_qgroup, old_w = ctx->frag_wg_per_cu;
    double best = 1e300, def_ms = 0;
    int best_g = old_g, best_w = old_w;
    try {
      for (int g : groups) {
        for (int w : wgs) {
          ctx->eri_qgroup = g;
          ctx->frag_wg_per_cu = w;
          enqueue_batch(ctx, ctx->sync_ws, prec, fr, false);     // warm-up (sizes the workspace)
          double ms = 1e300;
          for (int rep = 0; rep < 2; ++rep) {
            HIPCHK(hipEventRecord(e0, ctx->stream));
            enqueue_batch(ctx, ctx->sync_ws, prec, fr, false);
            HIPCHK(hipEventRecord(e1, ctx->stream));
            HIPCHK(hipEventSynchronize(e1));
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, (double)t);
          }
          if (g == def_g && w == FRAG_WG_PER_CU) def_ms = ms;
          if (ms < best) { best = ms; best_g = g; best_w = w; }
        }
      }
    } catch (...) {
      ctx->eri_qgroup = old_g;
      ctx->frag_wg_per_cu = old_w;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->eri_qgroup = best_g;
    ctx->frag_wg_per_cu = best_w;
    if (report) {
      report->eri_qgroup = best_g;
      report->wg_per_cu = best_w;
      report->ms = best;
      report->ms_default = def_ms;
      report->n_tried = (int32_t)(groups.size() * 4);
    }
  });
}

isdf_status isdf_serve_start(isdf_ctx ctx, int32_t max_inflight, int32_t max_batch, int64_t budget_bytes) {
  return guarded(ctx, [&] {
    if (ctx->serving) throw Fail{ISDF_E_STATE, "already serving"};
    if (max_inflight < 1 || max_inflight > 8 || max_batch < 1 || budget_bytes <= 0)
      throw Fail{ISDF_E_INVALID, "bad serving parameters"};
    ctx->max_inflight = max_inflight;
    ctx->max_batch = max_batch;
    ctx->budget = budget_bytes;
    ctx->stop = false;
    for (Workspace* w : ctx->ws_pool) delete w;
    ctx->ws_pool.clear();
    for (int i = 0; i < max_inflight; ++i) {
      Workspace* w = new Workspace();
      ctx->ws_pool.push_back(w);
      HIPCHK(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
      w->own_stream = true;
      HIPCHK(hipEventCreateWithFlags(&w->done, hipEventDisableTiming));
    }
    // every workspace holds its share of the budget from the start, so that
    // admitting a batch allocates nothing (a refit hands the memory to the
    // fit and the next Coulomb kernel takes it back)
    try {
      reserve_workspaces(ctx);
    } catch (...) {
      for (Workspace* w : ctx->ws_pool) delete w;
      ctx->ws_pool.clear();
      throw;
    }
    ctx->serving = true;
    ctx->worker = std::thread([ctx] {
      (void)hipSetDevice(ctx->device);
      serve_loop(ctx);
    });
  });
}

isdf_status isdf_submit(isdf_ctx ctx, const isdf_request* req, uint64_t* ticket) {
  return isdf_submit_n(ctx, 1, req, ticket);
}

isdf_status isdf_submit_n(isdf_ctx ctx, int32_t n, const isdf_request* reqs, uint64_t* tickets) {
  if (!ctx) return ISDF_E_INVALID;
  if (n < 1 || !reqs || !tickets) return fail(ctx, ISDF_E_INVALID, "bad request list");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!ctx->serving || ctx->stop) return fail(ctx, ISDF_E_STATE, "not serving");
  if (ctx->queue.size() + n > 100000) return fail(ctx, ISDF_E_BUSY, "request queue full");
  for (int i = 0; i < n; ++i) {
    const isdf_request* req = reqs + i;
    if (req->n_f < 1 || req->n_f > ctx->nk * ctx->norb || !req->C || !req->eri ||
        req->prec < ISDF_FP64 || req->prec > ISDF_MIXED_BF16)
      return fail(ctx, ISDF_E_INVALID, "bad request " + std::to_string(i));
    const bool host_out = !(req->flags & ISDF_FRAG_DEVICE);
    if ((long long)request_bytes(ctx, req->n_f, host_out, req->prec) > ctx->budget / ctx->max_inflight)
      return fail(ctx, ISDF_E_NOMEM, "request " + std::to_string(i) + " exceeds the per-batch memory budget");
  }
  const double t0 = now_s();
  for (int i = 0; i < n; ++i) {
    const uint64_t t = ctx->next_ticket++;
    Request r;
    r.req = reqs[i];
    r.t_submit = t0;
    ctx->reqs.emplace(t, r);
    // admission order: after every queued request of the same or a higher
    // priority (FIFO among equals)
    auto pos = ctx->queue.end();
    while (pos != ctx->queue.begin()) {
      auto prev = std::prev(pos);
      auto it = ctx->reqs.find(*prev);
      if (it != ctx->reqs.end() && it->second.req.priority >= reqs[i].priority) break;
      pos = prev;
    }
    ctx->queue.insert(pos, t);
    tickets[i] = t;
  }
  ctx->cv.notify_all();
  return ISDF_OK;
}

isdf_status isdf_poll(isdf_ctx ctx, uint64_t ticket, int32_t* state, double* latency_s) {
  if (!ctx) return ISDF_E_INVALID;
  if (!state) return fail(ctx, ISDF_E_INVALID, "null state");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->reqs.find(ticket);
  if (it == ctx->reqs.end()) return fail(ctx, ISDF_E_NOTFOUND, "unknown ticket");
  *state = it->second.state;
  if (latency_s) {
    const Request& r = it->second;
    *latency_s = (r.state == ISDF_REQ_DONE || r.state == ISDF_REQ_FAILED) ? r.t_done - r.t_submit : -1.0;
  }
  return ISDF_OK;
}

isdf_status isdf_cancel(isdf_ctx ctx, uint64_t ticket) {
  if (!ctx) return ISDF_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->reqs.find(ticket);
  if (it == ctx->reqs.end()) return fail(ctx, ISDF_E_NOTFOUND, "unknown ticket");
  if (it->second.state != ISDF_REQ_QUEUED)
    return fail(ctx, ISDF_E_STATE, "request already running or finished");
  it->second.state = ISDF_REQ_CANCELLED;
  return ISDF_OK;
}

isdf_status isdf_serve_stop(isdf_ctx ctx) {
  if (!ctx) return ISDF_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->serving) return ISDF_OK;
    ctx->stop = true;
    ctx->cv.notify_all();
  }
  if (ctx->worker.joinable()) ctx->worker.join();
  ctx->serving = false;
  for (Workspace* w : ctx->ws_pool) delete w;
  ctx->ws_pool.clear();
  if (!ctx->serve_err.empty()) return fail(ctx, ISDF_E_DEVICE, ctx->serve_err);
  return ISDF_OK;
}

isdf_status isdf_stats(isdf_ctx ctx, char* json, int64_t cap) {
  if (!ctx) return ISDF_E_INVALID;
  if (!json || cap <= 0) return fail(ctx, ISDF_E_INVALID, "bad buffer");
  std::string s = "{\"n_k\":" + std::to_string(ctx->nk) + ",\"n_g\":" + std::to_string(ctx->ng) +
                  ",\"n_orb\":" + std::to_string(ctx->norb) + ",\"n_ip\":" + std::to_string(ctx->nip) +
                  ",\"r_tile\":" + std::to_string(ctx->rc) + ",\"ip_tile\":" + std::to_string(ctx->ri) +
                  ",\"classes\":" + std::to_string(ctx->nh) + ",\"q_batch\":" + std::to_string(ctx->qb) +
                  ",\"w_factor\":" + (ctx->wfac ? "true" : "false") +
                  ",\"eri_qgroup\":" + std::to_string(ctx->eri_qgroup) +
                  ",\"eri_qgroup_initial\":" + std::to_string(ctx->eri_qgroup0) +
                  ",\"wg_per_cu\":" + std::to_string(ctx->frag_wg_per_cu) + ",\"rank\":[";
  // per q (the class of q or of -q; the factor of conj Pi has the same rank)
  if (!ctx->rank_h.empty())
    for (int q = 0; q < ctx->nk; ++q) {
      bool cj;
      s += (q ? "," : "") + std::to_string(ctx->rank_h[class_slot(ctx, q, &cj)]);
    }
  s += "],\"stage_ms\":{";
  bool first = true;
  for (auto& kv : ctx->timer.ms) {
    char b[64];
    snprintf(b, sizeof(b), "%.6f", kv.second);
    s += std::string(first ? "" : ",") + "\"" + kv.first + "\":" + b;
    first = false;
  }
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    s += "},\"served\":" + std::to_string(ctx->served) + ",\"batches\":" + std::to_string(ctx->batches) + "}";
  }
  strncpy(json, s.c_str(), (size_t)cap - 1);
  json[cap - 1] = 0;
  return ISDF_OK;
}

isdf_status isdf_stage_total(isdf_ctx ctx, const char* name, double* ms, int64_t* count) {
  if (!ctx) return ISDF_E_INVALID;
  if (!name || !ms || !count) return fail(ctx, ISDF_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->totals.find(name);
  *ms = it == ctx->totals.end() ? 0.0 : it->second.first;
  *count = it == ctx->totals.end() ? 0 : it->second.second;
  return ISDF_OK;
}

isdf_status isdf_stage_reset(isdf_ctx ctx) {
  if (!ctx) return ISDF_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->totals.clear();
  return ISDF_OK;
}

double isdf_stage_ms(isdf_ctx ctx, const char* name) {
  if (!ctx || !name) return -1.0;
  auto it = ctx->timer.ms.find(name);
  return it == ctx->timer.ms.end() ? -1.0 : (double)it->second;
}

isdf_status isdf_destroy(isdf_ctx ctx) {
  if (!ctx) return ISDF_E_INVALID;
  (void)isdf_serve_stop(ctx);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  if (ctx->aux2) {
    (void)hipStreamSynchronize(ctx->aux2);
    (void)hipStreamDestroy(ctx->aux2);
  }
  for (int b = 0; b < 2; ++b) {
    if (ctx->ev_rt[b]) (void)hipEventDestroy(ctx->ev_rt[b]);
    if (ctx->ev_kc[b]) (void)hipEventDestroy(ctx->ev_kc[b]);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->ev_pinv) (void)hipEventDestroy(ctx->ev_pinv);
  delete ctx;
  return ISDF_OK;
}

// Device buffer for a synchronous call; when the device is full, the idle
// workspace of synchronous fragment calls is handed back and the allocation
// tried once more.
static void alloc_reclaim(isdf_ctx c, DevBuf& b, size_t bytes) {
  try {
    b.alloc(bytes);
  } catch (const Fail& f) {
    if (f.st != ISDF_E_NOMEM) throw;
    HIPCHK(hipStreamSynchronize(c->stream));
    c->sync_ws.mem.release();
    b.alloc(bytes);
  }
}

isdf_status isdf_hf_jk(isdf_ctx ctx, const void* dm, void* j_out, void* k_out, uint32_t flags) {
  return guarded(ctx, [&] {
    if (!dm || (!j_out && !k_out)) throw Fail{ISDF_E_INVALID, "null density matrix or no output"};
    if (!ctx->kernel_ready) throw Fail{ISDF_E_STATE, "isdf_coulomb_kernel must run before isdf_hf_jk"};
    if (k_out && ctx->nk > 2048)
      throw Fail{ISDF_E_INVALID, "the exchange convolution holds two k columns in LDS: at most 2048 k points"};
    isdf_ctx c = ctx;
    hipStream_t s = c->stream;
    const int nk = c->nk, norb = c->norb, nip = c->nip;
    const bool dev = (flags & ISDF_HF_DEVICE) != 0;
    if (dev) {
      for (const void* ptr : {dm, (const void*)j_out, (const void*)k_out}) {
        if (!ptr) continue;
        hipPointerAttribute_t at;
        if (hipPointerGetAttributes(&at, ptr) != hipSuccess || at.type != hipMemoryTypeDevice) {
          (void)hipGetLastError();
          throw Fail{ISDF_E_INVALID, "ISDF_HF_DEVICE buffers must be device memory"};
        }
      }
    }
    const size_t mb = (size_t)nk * norb * norb * sizeof(cplx);
    const long long nn = (long long)nip * nip, on = (long long)norb * nip, oo = (long long)norb * norb;
    DevBuf dmd, jd, kd, rho, zb, nv, vv;
    const cplx* P = (const cplx*)dm;
    cplx* J = (cplx*)j_out;
    cplx* K = (cplx*)k_out;
    if (!dev) {
      alloc_reclaim(c, dmd, mb);
      HIPCHK(hipMemcpyAsync(dmd.p, dm, mb, hipMemcpyHostToDevice, s));
      P = dmd.as<cplx>();
      if (J) { alloc_reclaim(c, jd, mb); J = jd.as<cplx>(); }
      if (K) { alloc_reclaim(c, kd, mb); K = kd.as<cplx>(); }
    }
    alloc_reclaim(c, rho, sizeof(cplx) * (size_t)nk * nn);
    alloc_reclaim(c, zb, sizeof(cplx) * (size_t)nk * on);
    c->arena.reset(s);
    c->arena.reserve(((size_t)1 << 20) + (size_t)nk * sizeof(int));
    const cplx* xt = c->xt.as<cplx>();
    // rho^k_{IJ} = sum_{la sg} X^k_{I la} P^k_{la sg} conj(X^k_{J sg}) as
    // Z^k = P^k X^{k H} ([la][J]) and rho^k = X^k Z^k, FP64 MFMA
    c->timer.begin("hf_rho", s);
    {
      std::vector<GemmDesc> d(1);
      d[0] = mkdesc(P, norb, xt, nip, zb.as<cplx>(), nip, norb, nip, norb);
      d[0].batch = nk;
      d[0].sA_bat = oo;
      d[0].sB_bat = d[0].sC_bat = on;
      run_gemm(c->arena, 0, GEMM_B_KN | GEMM_B_CONJ, d, s);
    }
    {
      std::vector<GemmDesc> d(1);
      d[0] = mkdesc(xt, nip, zb.as<cplx>(), nip, rho.as<cplx>(), nip, nip, nip, norb);
      d[0].batch = nk;
      d[0].sA_bat = d[0].sB_bat = on;
      d[0].sC_bat = nn;
      run_gemm(c->arena, 0, GEMM_A_KM | GEMM_B_KN, d, s);
    }
    c->timer.end("hf_rho", s);
    if (J) {
      // J^k_{mu nu} = N_k^-1 sum_I conj(X^k_{I mu}) X^k_{I nu} (W^0 n)_I,
      // n_J = sum_k rho^k_{JJ} (before the exchange convolution reuses rho)
      c->timer.begin("hf_j", s);
      alloc_reclaim(c, nv, sizeof(cplx) * nip);
      alloc_reclaim(c, vv, sizeof(cplx) * nip);
      HIPCHK(hf_diag_sum_launch(rho.as<cplx>(), nk, nip, nv.as<cplx>(), s));
      bool cj;
      const int h0 = class_slot(c, 0, &cj);
      HIPCHK(hf_matvec_launch(c->w.as<cplx>() + (long long)h0 * nn, cj ? 1 : 0, nv.as<cplx>(), nip, 1.0 / nk,
                              vv.as<cplx>(), s));
      HIPCHK(hf_scale_launch(xt, vv.as<cplx>(), (long long)nk * norb, nip, zb.as<cplx>(), s));
      std::vector<NtDesc> d(1);
      d[0] = mknt(xt, nip, zb.p, nip, J, norb, norb, norb, nip);
      d[0].batch = nk;
      d[0].sA_bat = d[0].sB_bat = on;
      d[0].sC_bat = oo;
      run_nt(c->arena, 0, 1, d, s);
      c->timer.end("hf_j", s);
    }
    if (K) {
      // M^k = N_k^-1 sum_q W^q o rho^{k+q} by the convolution over k (eq. (10)),
      // in place, then K^k = X^{k H} M^k X^k as two NT products
      c->timer.begin("hf_kconv", s);
      std::vector<int> wsel(nk);
      for (int q = 0; q < nk; ++q) {
        bool cq;
        const int h = class_slot(c, q, &cq);
        wsel[q] = (h << 1) | (cq ? 1 : 0);
      }
      const int* wsel_d = c->arena.put(wsel.data(), wsel.size(), s);
      XconvArgs a;
      memset(&a, 0, sizeof(a));
      a.rho = rho.as<cplx>();
      a.w = c->w.as<cplx>();
      a.wsel = wsel_d;
      a.n_elem = nn;
      a.m1 = c->m[0];
      a.m2 = c->m[1];
      a.m3 = c->m[2];
      a.scale = 1.0 / ((double)nk * nk);
      HIPCHK(xconv_launch(a, s));
      c->timer.end("hf_kconv", s);
      c->timer.begin("hf_k", s);
      {
        // Zt^k[nu][I] = sum_J X^k_{J nu} M^k_{IJ}
        std::vector<NtDesc> d(1);
        d[0] = mknt(xt, nip, rho.p, nip, zb.p, nip, norb, nip, nip);
        d[0].batch = nk;
        d[0].sA_bat = on;
        d[0].sB_bat = nn;
        d[0].sC_bat = on;
        run_nt(c->arena, 0, 0, d, s);
      }
      {
        // K^k[mu][nu] = sum_I conj(X^k_{I mu}) Zt^k[nu][I]
        std::vector<NtDesc> d(1);
        d[0] = mknt(xt, nip, zb.p, nip, K, norb, norb, norb, nip);
        d[0].batch = nk;
        d[0].sA_bat = d[0].sB_bat = on;
        d[0].sC_bat = oo;
        run_nt(c->arena, 0, 1, d, s);
      }
      c->timer.end("hf_k", s);
    }
    if (!dev) {
      if (j_out) HIPCHK(hipMemcpyAsync(j_out, J, mb, hipMemcpyDeviceToHost, s));
      if (k_out) HIPCHK(hipMemcpyAsync(k_out, K, mb, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    std::lock_guard<std::mutex> lk(c->mu);
    c->timer.collect(&c->totals);
  });
}

// The polarisabilities at one tau (eqs. (13)-(15)): Go^k = Yo e^{tau (e_i - mu)}
// Yo^H and Gv^k = Yv e^{-tau (e_a - mu)} Yv^H into bo, bv (Hermitian FP64
// MFMA products of the scaled orbitals at the points), then chi^q into bv and
// chit^q into bo, one q per class in class order, by the convolution over k.
static void tau_polarisabilities(isdf_ctx c, const cplx* y, const double* ed, int n_mo, int n_occ, double tau,
                                 double mu, cplx* yo, cplx* yv, cplx* bo, cplx* bv) {
  hipStream_t s = c->stream;
  const int nk = c->nk, nip = c->nip, nvir = n_mo - n_occ;
  const long long nn = (long long)nip * nip;
  c->timer.begin("mp2_green", s);
  HIPCHK(mp2_scale_launch(y, ed, nk, nip, n_mo, n_occ, tau, mu, yo, yv, s));
  for (int which = 0; which < 2; ++which) {
    const int kk = which == 0 ? n_occ : nvir;
    void* src = which == 0 ? (void*)yo : (void*)yv;
    std::vector<NtDesc> d(1);
    d[0] = mknt(src, kk, src, kk, which == 0 ? (void*)bo : (void*)bv, nip, nip, nip, kk);
    d[0].batch = nk;
    d[0].sA_bat = d[0].sB_bat = (long long)nip * kk;
    d[0].sC_bat = nn;
    d[0].herm = 1;
    run_nt(c->arena, 0, 2, d, s);
  }
  c->timer.end("mp2_green", s);
  c->timer.begin("mp2_pconv", s);
  PconvArgs a;
  memset(&a, 0, sizeof(a));
  a.gv = bv;
  a.go = bo;
  a.n_elem = nn;
  a.m1 = c->m[0];
  a.m2 = c->m[1];
  a.m3 = c->m[2];
  a.scale = 1.0 / ((double)nk * nk);
  a.qslot = c->qmap.as<int>();
  HIPCHK(pconv_launch(a, s));
  c->timer.end("mp2_pconv", s);
}

// Shared checks of the correlation-energy calls; returns the chemical
// potential between the occupied and virtual energies.
static double check_mo(isdf_ctx c, const void* mo_coeff, const double* mo_energy, int n_mo, int n_occ, int n_tau,
                       const double* tau, const double* weight, uint32_t flags, const char* name) {
  // weight: the time weights (MP2) or the time points again (dRPA, whose
  // transform is checked by the caller)
  if (!mo_coeff || !mo_energy || !tau || !weight) throw Fail{ISDF_E_INVALID, "null argument"};
  if (n_mo < 2 || n_mo > c->norb || n_occ < 1 || n_occ >= n_mo)
    throw Fail{ISDF_E_INVALID, "need 1 <= n_occ < n_mo <= n_orb"};
  if (n_tau < 1 || n_tau > 4096) throw Fail{ISDF_E_INVALID, "n_tau must be 1..4096"};
  for (int n = 0; n < n_tau; ++n)
    if (!(tau[n] >= 0.0) || !std::isfinite(tau[n]) || !std::isfinite(weight[n]))
      throw Fail{ISDF_E_INVALID, "tau must be finite and >= 0, weights finite"};
  if (!c->kernel_ready) throw Fail{ISDF_E_STATE, std::string("isdf_coulomb_kernel must run before ") + name};
  if (c->nk > 2048)
    throw Fail{ISDF_E_INVALID, "the polarisability convolution holds two k columns in LDS: at most 2048 k points"};
  double homo = -INFINITY, lumo = INFINITY;
  for (int k = 0; k < c->nk; ++k)
    for (int p = 0; p < n_mo; ++p) {
      const double e = mo_energy[(long long)k * n_mo + p];
      if (!std::isfinite(e)) throw Fail{ISDF_E_INVALID, "non-finite orbital energy"};
      if (p < n_occ) homo = std::max(homo, e);
      else lumo = std::min(lumo, e);
    }
  if (!(homo < lumo)) throw Fail{ISDF_E_INVALID, "occupied and virtual energies overlap (no gap)"};
  if (flags & 0x1u) {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, mo_coeff) != hipSuccess || at.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      throw Fail{ISDF_E_INVALID, "device-flagged coefficients must be device memory"};
    }
  }
  return 0.5 * (homo + lumo);
}

isdf_status isdf_sos_mp2(isdf_ctx ctx, const void* mo_coeff, const double* mo_energy, int32_t n_mo, int32_t n_occ,
                         int32_t n_tau, const double* tau, const double* weight, double* integrand_out,
                         double* class_out, double* e_os_out, uint32_t flags) {
  return guarded(ctx, [&] {
    isdf_ctx c = ctx;
    if (!e_os_out) throw Fail{ISDF_E_INVALID, "null argument"};
    // chemical potential between the occupied and virtual energies (it cancels)
    const double mu = check_mo(c, mo_coeff, mo_energy, n_mo, n_occ, n_tau, tau, weight, flags, "isdf_sos_mp2");
    const int nk = c->nk, norb = c->norb, nip = c->nip, nh = c->nh, nvir = n_mo - n_occ;
    const bool dev = (flags & ISDF_MP2_DEVICE) != 0;
    hipStream_t s = c->stream;
    const long long nn = (long long)nip * nip;
    const int nblk = std::max(1, std::min(64, (2048 + nh - 1) / nh));
    DevBuf cd, ed, y, yo, yv, bo, bv, t1, part;
    const cplx* C = (const cplx*)mo_coeff;
    if (!dev) {
      alloc_reclaim(c, cd, sizeof(cplx) * (size_t)nk * norb * n_mo);
      HIPCHK(hipMemcpyAsync(cd.p, mo_coeff, sizeof(cplx) * (size_t)nk * norb * n_mo, hipMemcpyHostToDevice, s));
      C = cd.as<cplx>();
    }
    alloc_reclaim(c, ed, sizeof(double) * (size_t)nk * n_mo);
    HIPCHK(hipMemcpyAsync(ed.p, mo_energy, sizeof(double) * (size_t)nk * n_mo, hipMemcpyHostToDevice, s));
    alloc_reclaim(c, y, sizeof(cplx) * (size_t)nk * nip * n_mo);
    alloc_reclaim(c, yo, sizeof(cplx) * (size_t)nk * nip * n_occ);
    alloc_reclaim(c, yv, sizeof(cplx) * (size_t)nk * nip * nvir);
    alloc_reclaim(c, bo, sizeof(cplx) * (size_t)nk * nn);
    alloc_reclaim(c, bv, sizeof(cplx) * (size_t)nk * nn);
    alloc_reclaim(c, t1, sizeof(cplx) * (size_t)nh * nn);
    alloc_reclaim(c, part, sizeof(cplx) * (size_t)nh * nblk);
    const cplx* xt = c->xt.as<cplx>();
    // Y^k = X^k C^k (canonical orbitals at the interpolation points)
    c->arena.reset(s);
    c->arena.reserve((size_t)1 << 20);
    {
      std::vector<GemmDesc> d(1);
      d[0] = mkdesc(xt, nip, C, n_mo, y.as<cplx>(), n_mo, nip, n_mo, norb);
      d[0].batch = nk;
      d[0].sA_bat = (long long)norb * nip;
      d[0].sB_bat = (long long)norb * n_mo;
      d[0].sC_bat = (long long)nip * n_mo;
      run_gemm(c->arena, 0, GEMM_A_KM | GEMM_B_KN, d, s);
    }
    std::vector<cplx> ph((size_t)nh * nblk);
    double e_os = 0.0;
    for (int n = 0; n < n_tau; ++n) {
      c->arena.reset(s);
      c->arena.reserve((size_t)1 << 20);
      tau_polarisabilities(c, y.as<cplx>(), ed.as<double>(), n_mo, n_occ, tau[n], mu, yo.as<cplx>(),
                           yv.as<cplx>(), bo.as<cplx>(), bv.as<cplx>());
      // T1 = W chi, T2 = chit W (FP64 MFMA), tr[W chi W chit] = sum T1 o conj(T2)
      c->timer.begin("mp2_wchi", s);
      {
        std::vector<GemmDesc> d(1);
        d[0] = mkdesc(c->w.as<cplx>(), nip, bv.as<cplx>(), nip, t1.as<cplx>(), nip, nip, nip, nip);
        d[0].batch = nh;
        d[0].sA_bat = d[0].sB_bat = d[0].sC_bat = nn;
        run_gemm(c->arena, 0, GEMM_B_KN, d, s);
        std::vector<GemmDesc> d2(1);
        d2[0] = mkdesc(bo.as<cplx>(), nip, c->w.as<cplx>(), nip, bv.as<cplx>(), nip, nip, nip, nip);
        d2[0].batch = nh;
        d2[0].sA_bat = d2[0].sB_bat = d2[0].sC_bat = nn;
        run_gemm(c->arena, 0, GEMM_B_KN, d2, s);
      }
      c->timer.end("mp2_wchi", s);
      c->timer.begin("mp2_trace", s);
      HIPCHK(mp2_dot_launch(t1.as<cplx>(), bv.as<cplx>(), nn, nh, nblk, part.as<cplx>(), s));
      c->timer.end("mp2_trace", s);
      HIPCHK(hipMemcpyAsync(ph.data(), part.p, sizeof(cplx) * ph.size(), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      // classes {q, -q} with q != -q stand for two equal-real-part terms
      double f = 0.0;
      for (int h = 0; h < nh; ++h) {
        double re = 0.0;
        for (int b = 0; b < nblk; ++b) re += ph[(size_t)h * nblk + b].x;
        const double term = (c->hself_h[h] ? 1.0 : 2.0) * re / nk;
        if (class_out) class_out[(size_t)n * nh + h] = term;
        f += term;
      }
      if (integrand_out) integrand_out[n] = f;
      e_os -= weight[n] * f;
    }
    *e_os_out = e_os;
    std::lock_guard<std::mutex> lk(c->mu);
    c->timer.collect(&c->totals);
  });
}

isdf_status isdf_drpa(isdf_ctx ctx, const void* mo_coeff, const double* mo_energy, int32_t n_mo, int32_t n_occ,
                      int32_t n_tau, const double* tau, int32_t n_omega, const double* omega_weight,
                      const void* transform, double* integrand_out, double* class_out, double* e_drpa_out,
                      double* e_second_out, uint32_t flags) {
  return guarded(ctx, [&] {
    isdf_ctx c = ctx;
    if (!e_drpa_out || !omega_weight || !transform) throw Fail{ISDF_E_INVALID, "null argument"};
    if (n_omega < 1 || n_omega > 1024) throw Fail{ISDF_E_INVALID, "n_omega must be 1..1024"};
    const cplx* gam = (const cplx*)transform;
    for (int m = 0; m < n_omega; ++m) {
      if (!std::isfinite(omega_weight[m])) throw Fail{ISDF_E_INVALID, "frequency weights must be finite"};
      for (int n = 0; n < std::max(n_tau, 0); ++n) {
        const cplx g = gam[(size_t)m * n_tau + n];
        if (!std::isfinite(g.x) || !std::isfinite(g.y)) throw Fail{ISDF_E_INVALID, "non-finite transform entry"};
      }
    }
    const double mu = check_mo(c, mo_coeff, mo_energy, n_mo, n_occ, n_tau, tau, tau, flags, "isdf_drpa");
    const int nk = c->nk, norb = c->norb, nip = c->nip, nh = c->nh, nvir = n_mo - n_occ;
    const bool dev = (flags & ISDF_DRPA_DEVICE) != 0;
    hipStream_t s = c->stream;
    const long long nn = (long long)nip * nip, hn = (long long)nh * nn;
    const int ntile = drpa_trace2_tiles(nip);
    DevBuf cd, ed, y, yo, yv, bo, bv, pm, gm, lt, perm, rank, dmax, flag, tr, tr2, ld, ph, chiw;
    const cplx* C = (const cplx*)mo_coeff;
    if (!dev) {
      alloc_reclaim(c, cd, sizeof(cplx) * (size_t)nk * norb * n_mo);
      HIPCHK(hipMemcpyAsync(cd.p, mo_coeff, sizeof(cplx) * (size_t)nk * norb * n_mo, hipMemcpyHostToDevice, s));
      C = cd.as<cplx>();
    }
    alloc_reclaim(c, ed, sizeof(double) * (size_t)nk * n_mo);
    HIPCHK(hipMemcpyAsync(ed.p, mo_energy, sizeof(double) * (size_t)nk * n_mo, hipMemcpyHostToDevice, s));
    alloc_reclaim(c, y, sizeof(cplx) * (size_t)nk * nip * n_mo);
    alloc_reclaim(c, yo, sizeof(cplx) * (size_t)nk * nip * n_occ);
    alloc_reclaim(c, yv, sizeof(cplx) * (size_t)nk * nip * nvir);
    alloc_reclaim(c, bo, sizeof(cplx) * (size_t)nk * nn);
    alloc_reclaim(c, bv, sizeof(cplx) * (size_t)nk * nn);
    alloc_reclaim(c, pm, sizeof(cplx) * (size_t)hn);
    alloc_reclaim(c, gm, sizeof(cplx) * (size_t)hn);
    alloc_reclaim(c, lt, sizeof(cplx) * (size_t)hn);
    alloc_reclaim(c, perm, sizeof(int) * (size_t)nh * nip);
    alloc_reclaim(c, rank, sizeof(int) * (size_t)nh);
    alloc_reclaim(c, dmax, sizeof(double) * (size_t)nh);
    alloc_reclaim(c, flag, sizeof(int) * (size_t)nh);
    alloc_reclaim(c, tr, sizeof(cplx) * (size_t)nh);
    alloc_reclaim(c, tr2, sizeof(cplx) * (size_t)nh * ntile);
    alloc_reclaim(c, ld, sizeof(double) * (size_t)nh);
    alloc_reclaim(c, ph, sizeof(cplx) * (size_t)n_omega);
    // frequency polarisabilities of as many frequencies at once as fit in 90 %
    // of the free device memory (the time loop runs once per batch)
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    const long long per_w = hn * (long long)sizeof(cplx);
    int nbw = (int)std::min<long long>(n_omega, (long long)(0.9 * (double)fr) / per_w);
    if (nbw < 1) {
      HIPCHK(hipStreamSynchronize(s));
      c->sync_ws.mem.release();
      HIPCHK(hipMemGetInfo(&fr, &tot));
      nbw = (int)std::min<long long>(n_omega, (long long)(0.9 * (double)fr) / per_w);
    }
    if (nbw < 1) throw Fail{ISDF_E_NOMEM, "no room for one frequency of polarisabilities"};
    alloc_reclaim(c, chiw, (size_t)nbw * per_w);
    const cplx* xt = c->xt.as<cplx>();
    c->arena.reset(s);
    c->arena.reserve((size_t)1 << 20);
    {
      std::vector<GemmDesc> d(1);
      d[0] = mkdesc(xt, nip, C, n_mo, y.as<cplx>(), n_mo, nip, n_mo, norb);
      d[0].batch = nk;
      d[0].sA_bat = (long long)norb * nip;
      d[0].sB_bat = (long long)norb * n_mo;
      d[0].sC_bat = (long long)nip * n_mo;
      run_gemm(c->arena, 0, GEMM_A_KM | GEMM_B_KN, d, s);
    }
    std::vector<cplx> h_tr(nh), h_tr2((size_t)nh * ntile), h_ph(nbw);
    std::vector<double> h_ld(nh);
    double e_rpa = 0.0, e_2 = 0.0;
    for (int m0 = 0; m0 < n_omega; m0 += nbw) {
      const int nb = std::min(nbw, n_omega - m0);
      // chi^q(iw_m) = -sum_n tw_n [exp(i w_m tau_n) chi^q(tau_n) + exp(-i w_m tau_n) chit^q(tau_n)]
      HIPCHK(zero_launch(chiw.as<cplx>(), (long long)nb * hn, s));
      for (int n = 0; n < n_tau; ++n) {
        c->arena.reset(s);
        c->arena.reserve((size_t)1 << 20);
        tau_polarisabilities(c, y.as<cplx>(), ed.as<double>(), n_mo, n_occ, tau[n], mu, yo.as<cplx>(),
                             yv.as<cplx>(), bo.as<cplx>(), bv.as<cplx>());
        for (int m = 0; m < nb; ++m) h_ph[m] = gam[(size_t)(m0 + m) * n_tau + n];
        HIPCHK(hipMemcpyAsync(ph.p, h_ph.data(), sizeof(cplx) * nb, hipMemcpyHostToDevice, s));
        c->timer.begin("drpa_accum", s);
        HIPCHK(drpa_accum_launch(bv.as<cplx>(), bo.as<cplx>(), hn, ph.as<cplx>(), nb, chiw.as<cplx>(), s));
        c->timer.end("drpa_accum", s);
        HIPCHK(hipStreamSynchronize(s));   // h_ph is reused by the next tau
      }
      for (int m = 0; m < nb; ++m) {
        c->arena.reset(s);
        c->arena.reserve((size_t)1 << 20);
        cplx* chi = chiw.as<cplx>() + (long long)m * hn;
        // P = chi W; tr P, tr P^2; A = 1 - P; G = A^H A = L L^H; ln|det A|^2 = ln det G
        c->timer.begin("drpa_p", s);
        {
          std::vector<GemmDesc> d(1);
          d[0] = mkdesc(chi, nip, c->w.as<cplx>(), nip, pm.as<cplx>(), nip, nip, nip, nip);
          d[0].batch = nh;
          d[0].sA_bat = d[0].sB_bat = d[0].sC_bat = nn;
          run_gemm(c->arena, 0, GEMM_B_KN, d, s);
        }
        HIPCHK(drpa_trace_launch(pm.as<cplx>(), nip, nh, tr.as<cplx>(), s));
        HIPCHK(drpa_trace2_launch(pm.as<cplx>(), nip, nh, tr2.as<cplx>(), s));
        HIPCHK(drpa_one_minus_launch(pm.as<cplx>(), nip, nh, s));
        c->timer.end("drpa_p", s);
        c->timer.begin("drpa_logdet", s);
        {
          std::vector<GemmDesc> d(1);
          d[0] = mkdesc(pm.as<cplx>(), nip, pm.as<cplx>(), nip, gm.as<cplx>(), nip, nip, nip, nip);
          d[0].batch = nh;
          d[0].sA_bat = d[0].sB_bat = d[0].sC_bat = nn;
          d[0].herm = 1;
          run_gemm(c->arena, 0, GEMM_A_KM | GEMM_B_KN | GEMM_A_CONJ, d, s);
        }
        chol_blocked(c->arena, gm.as<cplx>(), pm.as<cplx>(), lt.as<cplx>(), perm.as<int>(), rank.as<int>(),
                     dmax.as<double>(), flag.as<int>(), nip, nh, 0.0, s);
        HIPCHK(drpa_logdet_launch(pm.as<cplx>(), flag.as<int>(), nip, nh, ld.as<double>(), s));
        c->timer.end("drpa_logdet", s);
        HIPCHK(hipMemcpyAsync(h_tr.data(), tr.p, sizeof(cplx) * nh, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h_tr2.data(), tr2.p, sizeof(cplx) * h_tr2.size(), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h_ld.data(), ld.p, sizeof(double) * nh, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        // per class: Re ln det(1 - P) + Re tr P and -1/2 Re tr P^2; a class with
        // q != -q stands for two equal real parts
        double f = 0.0, f2 = 0.0;
        for (int h = 0; h < nh; ++h) {
          if (!std::isfinite(h_ld[h]))
            throw Fail{ISDF_E_NUMERIC, "1 - chi W singular at frequency point " + std::to_string(m0 + m) +
                                           ", q = " + std::to_string(c->hq_h[h])};
          double t2 = 0.0;
          for (int t = 0; t < ntile; ++t) t2 += h_tr2[(size_t)h * ntile + t].x;
          const double wt = c->hself_h[h] ? 1.0 : 2.0;
          const double term = wt * (0.5 * h_ld[h] + h_tr[h].x);
          if (class_out) class_out[(size_t)(m0 + m) * nh + h] = term / (M_PI * nk);
          f += term;
          f2 += wt * (-0.5 * t2);
        }
        f /= M_PI * nk;
        f2 /= M_PI * nk;
        if (integrand_out) integrand_out[m0 + m] = f;
        e_rpa += omega_weight[m0 + m] * f;
        e_2 += omega_weight[m0 + m] * f2;
      }
    }
    *e_drpa_out = e_rpa;
    if (e_second_out) *e_second_out = e_2;
    std::lock_guard<std::mutex> lk(c->mu);
    c->timer.collect(&c->totals);
  });
}

const char* isdf_last_error(isdf_ctx ctx) {
  if (!ctx) return t_create_err.empty() ? "null context" : t_create_err.c_str();
  return ctx->err.c_str();
}

isdf_status isdf_save(isdf_ctx ctx, const char* path) {
  return guarded(ctx, [&] {
    if (!path) throw Fail{ISDF_E_INVALID, "null path"};
    if (!ctx->kernel_ready) throw Fail{ISDF_E_STATE, "no Coulomb kernel to save (isdf_coulomb_kernel first)"};
    CkHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, kCkMagic, 8);
    h.version = 1;
    h.header_bytes = sizeof(CkHeader);
    for (int d = 0; d < 3; ++d) { h.grid[d] = ctx->n[d]; h.kmesh[d] = ctx->m[d]; }
    h.n_orb = ctx->norb;
    h.n_ip = ctx->nip;
    h.nh = ctx->nh;
    h.flags = ctx->flags & ~(uint32_t)ISDF_INPUT_DEVICE;
    memcpy(h.lattice, ctx->lattice, sizeof(h.lattice));
    h.payload_bytes = ck_payload_bytes(h);
    FILE* f = fopen(path, "wb");
    if (!f) throw Fail{ISDF_E_INVALID, std::string("cannot open ") + path + " for writing"};
    std::unique_ptr<FILE, int (*)(FILE*)> guard(f, fclose);
    if (fwrite(&h, sizeof(h), 1, f) != 1) throw Fail{ISDF_E_INVALID, "write failed"};
    uint64_t sum = kFnvInit;
    auto put_host = [&](const void* p, size_t n) {
      if (n && fwrite(p, 1, n, f) != n) throw Fail{ISDF_E_INVALID, "write failed"};
      sum = fnv1a(sum, (const unsigned char*)p, n);
    };
    // device arrays go through one pinned staging buffer
    PinnedBuf stage;
    const size_t chunk = (size_t)64 << 20;
    stage.ensure(chunk);
    auto put_dev = [&](const void* dp, size_t n) {
      for (size_t o = 0; o < n; o += chunk) {
        const size_t b = std::min(chunk, n - o);
        HIPCHK(hipMemcpyAsync(stage.p, (const char*)dp + o, b, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        put_host(stage.p, b);
      }
    };
    HIPCHK(hipStreamSynchronize(ctx->stream));
    put_dev(ctx->ip.p, 4ull * ctx->nip);
    put_host(ctx->rank_h.data(), 4ull * ctx->nh);
    put_dev(ctx->xt.p, 16ull * ctx->nk * ctx->norb * ctx->nip);
    put_dev(ctx->pi.p, 16ull * ctx->nh * ctx->nip * ctx->nip);
    put_dev(ctx->w.p, 16ull * ctx->nh * ctx->nip * ctx->nip);
    h.checksum = sum;
    if (fseek(f, 0, SEEK_SET) != 0 || fwrite(&h, sizeof(h), 1, f) != 1) throw Fail{ISDF_E_INVALID, "write failed"};
  });
}

isdf_status isdf_load(isdf_ctx* out, const char* path, void* hip_stream) {
  t_create_err.clear();
  if (!out) { t_create_err = "null output handle"; return ISDF_E_INVALID; }
  *out = nullptr;
  if (!path) { t_create_err = "null path"; return ISDF_E_INVALID; }
  // the whole file is read and checked on the host before any device call
  CkHeader h;
  std::vector<unsigned char> pay;
  {
    FILE* f = fopen(path, "rb");
    if (!f) { t_create_err = std::string("cannot open ") + path; return ISDF_E_INVALID; }
    std::unique_ptr<FILE, int (*)(FILE*)> guard(f, fclose);
    if (fread(&h, sizeof(h), 1, f) != 1) { t_create_err = "truncated checkpoint header"; return ISDF_E_INVALID; }
    if (memcmp(h.magic, kCkMagic, 8) != 0) { t_create_err = "not an isdf checkpoint"; return ISDF_E_INVALID; }
    if (h.version != 1 || h.header_bytes != sizeof(CkHeader)) {
      t_create_err = "unsupported checkpoint version";
      return ISDF_E_INVALID;
    }
    if (const char* m = check_sizes(h.grid, h.kmesh, h.n_orb, h.n_ip)) {
      t_create_err = std::string("checkpoint sizes: ") + m;
      return ISDF_E_INVALID;
    }
    if (h.nh != classes_of(h.kmesh) || h.payload_bytes != ck_payload_bytes(h)) {
      t_create_err = "checkpoint sizes do not match its k mesh";
      return ISDF_E_INVALID;
    }
    try {
      pay.resize(h.payload_bytes);
    } catch (const std::bad_alloc&) {
      t_create_err = "host allocation failed";
      return ISDF_E_NOMEM;
    }
    if (fread(pay.data(), 1, pay.size(), f) != pay.size()) { t_create_err = "truncated checkpoint"; return ISDF_E_INVALID; }
    unsigned char extra;
    if (fread(&extra, 1, 1, f) != 0) { t_create_err = "trailing bytes after the checkpoint"; return ISDF_E_INVALID; }
  }
  if (fnv1a(kFnvInit, pay.data(), pay.size()) != h.checksum) {
    t_create_err = "checkpoint checksum mismatch";
    return ISDF_E_INVALID;
  }
  std::vector<int32_t> iph(h.n_ip), rk(h.nh);
  memcpy(iph.data(), pay.data(), 4ull * h.n_ip);
  memcpy(rk.data(), pay.data() + 4ull * h.n_ip, 4ull * h.nh);
  for (int r : rk)
    if (r < 1 || r > h.n_ip) { t_create_err = "checkpoint rank out of range"; return ISDF_E_INVALID; }
  isdf_ctx c = new (std::nothrow) isdf_ctx_s();
  if (!c) return ISDF_E_NOMEM;
  isdf_status st = guarded(c, [&] {
    check_ips(iph, (long long)h.grid[0] * h.grid[1] * h.grid[2]);
    setup_context(c, h.lattice, h.grid, h.kmesh, h.n_orb, h.n_ip, h.flags, hip_stream, false);
    const unsigned char* p = pay.data() + 4ull * h.n_ip + 4ull * h.nh;
    const size_t xb = 16ull * c->nk * c->norb * c->nip, mb = 16ull * c->nh * c->nip * c->nip;
    HIPCHK(hipMemcpy(c->ip.p, iph.data(), 4ull * h.n_ip, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->rank.p, rk.data(), 4ull * h.nh, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->xt.p, p, xb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->pi.p, p + xb, mb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->w.p, p + xb + mb, mb, hipMemcpyHostToDevice));
    c->rank_h = rk;
    // the operand copies of W for the fragment GEMMs
    c->arena.reset(c->stream);
    c->arena.reserve(((size_t)1 << 20) + (size_t)c->nh * 1024);
    operand_copies(c, nullptr, nullptr, c->stream);
    c->fitted = true;
    c->kernel_ready = true;
  });
  if (st != ISDF_OK) {
    t_create_err = c->err;
    delete c;
    return st;
  }
  *out = c;
  return ISDF_OK;
}

}  // extern "C"
