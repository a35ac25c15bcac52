// api.cpp -- the C ABI of libmpc (declared in include/mpc.h): context and
// workspace management, argument validation and the orchestration of the
// kernels for each protocol step.
#include <rocblas/rocblas.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <array>
#include <new>
#include <vector>
#include <atomic>
#include <mutex>

#include "internal.h"
#include "mpc.h"

using namespace mpc;

namespace {

// Written by whichever thread meets a HIP error, on any context.
std::atomic<int> g_last_hip_error{0};

#define HIPCHK(expr)                             \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) {                      \
      g_last_hip_error.store((int)_e);           \
      return MPC_E_HIP;                          \
    }                                            \
  } while (0)

#define CHK(expr)                 \
  do {                            \
    mpc_status _s = (expr);       \
    if (_s != MPC_OK) return _s;  \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Host staging slot for descriptor tables: a pinned buffer, its device mirror
// and an event marking the end of the call that last used it.
struct UploadSlot {
  void* host = nullptr;
  void* dev = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};
constexpr int kSlots = 16;

// Tile classes of a limb-form matrix product (the buckets the autotuner
// tunes separately): products of at most 32 rows or columns take the thin
// 32x128 or 128x32 tile when it leaves at most nine tenths of the 64x64
// tile's padded work (the thin tiles keep every wave at 32x32 outputs but
// share one operand among fewer waves).
enum { kBucketRegular = 0, kBucketThinM = 1, kBucketThinN = 2, kBuckets = 3 };
struct BucketScheds {
  TileSched s[kBuckets];
};

// Workspace of mpc_beaver_matmul_noalloc, for callers that cannot allocate:
// one array per device that loads the library, held until the process ends.
// In host code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, looked up once per device (with that device current)
// when the first context on it is created.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices];

// The device address of `scratch` on the current device `device`, or null
// (with the HIP error recorded) if it cannot be found.
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      g_last_hip_error.store((int)e);
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch[device] = ptr;
  }
  return g_scratch[device];
}

}  // namespace

struct mpc_ctx {
  int device = 0;
  int num_cu = 256;
  hipStream_t s[2] = {nullptr, nullptr};
  bool own[2] = {false, false};
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipStream_t side = nullptr;  // non-blocking stream for uploads made during capture
  uint64_t seed = 0;
  uint8_t* ws = nullptr;
  size_t ws_cap = 0;
  UploadSlot slots[kSlots];
  int next_slot = 0;
  int cur_slot = -1;
  bool capturing = false;
  // descriptor buffers made during the capture in progress; the graph that
  // capture becomes owns them and frees them when it is destroyed
  std::vector<void*> capture_allocs;
  mpc_stats stats{};
  // event timing of GEMM launches
  struct TimedLaunch {
    hipEvent_t start, stop;
    int form;
    double ring_macs;
  };
  bool profiling = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> event_pool;
  // limb GEMM tile schedule used when no tuned entry matches (for the regular
  // class; thin products take the thin tiles unless a default was set), and
  // the tuned schedules per class keyed by the hash of a matmul shape list
  TileSched sched_default{kLimbLds64x64, 8, 1};
  bool class_tiles = true;
  std::map<uint64_t, BucketScheds> tuned;
  // vendor BLAS handle of the fp64 limb form (created on first use)
  rocblas_handle blas = nullptr;
  // partial sums of split-K plain GEMMs (grown on demand)
  uint8_t* splitk = nullptr;
  size_t splitk_cap = 0;
  // instantiated graphs not yet destroyed: they hold workspace addresses, so
  // no buffer may move while any exists
  int live_graphs = 0;
  // this device's no-alloc workspace (`scratch`), or null if not found
  uint8_t* scratch = nullptr;
  // queue heads of the persistent limb GEMM (zeroed; each launch leaves them
  // zeroed, and all of this context's launches run on party 0's stream)
  unsigned* queue = nullptr;
};
// An instantiated graph, the context whose buffers it references and the
// descriptor buffers its kernels read.
struct mpc_graph {
  hipGraphExec_t exec;
  mpc_ctx* ctx;
  std::vector<void*> allocs;
};

namespace {

bool two_streams(const mpc_ctx* c) { return c->s[0] != c->s[1]; }

mpc_status set_device(mpc_ctx* c) {
  HIPCHK(hipSetDevice(c->device));
  return MPC_OK;
}

// Call protocol: every call is issued on party 0's stream.  Work local to
// party 1 is forked onto party 1's stream and joined back before the call
// returns, so both streams are idle-equivalent between calls and anything the
// caller ordered before the call on party 0's stream is visible to it.
// fork: party 1's stream waits for everything issued so far on party 0's.
mpc_status fork(mpc_ctx* c) {
  if (!two_streams(c)) return MPC_OK;
  HIPCHK(hipEventRecord(c->ev[0], c->s[0]));
  HIPCHK(hipStreamWaitEvent(c->s[1], c->ev[0], 0));
  return MPC_OK;
}

// join: party 0's stream waits for everything issued so far on party 1's.
mpc_status join(mpc_ctx* c) {
  if (!two_streams(c)) return MPC_OK;
  HIPCHK(hipEventRecord(c->ev[1], c->s[1]));
  HIPCHK(hipStreamWaitEvent(c->s[0], c->ev[1], 0));
  return MPC_OK;
}

mpc_status sync_all(mpc_ctx* c) {
  HIPCHK(hipStreamSynchronize(c->s[0]));
  if (two_streams(c)) HIPCHK(hipStreamSynchronize(c->s[1]));
  return MPC_OK;
}

// Makes the workspace at least `bytes`.  Growing frees the old buffer, so it
// first waits for both streams; it is refused while a graph is being captured.
mpc_status ensure_ws(mpc_ctx* c, size_t bytes) {
  if (bytes <= c->ws_cap) return MPC_OK;
  // a live graph (or one being captured) holds the current workspace address
  if (c->capturing || c->live_graphs > 0) return MPC_E_NOMEM;
  CHK(sync_all(c));
  if (c->ws) HIPCHK(hipFree(c->ws));
  c->ws = nullptr;
  c->ws_cap = 0;
  size_t cap = align_up(bytes + bytes / 4, 1 << 20);
  if (hipMalloc((void**)&c->ws, cap) != hipSuccess) {
    c->ws = nullptr;
    (void)hipGetLastError();
    return MPC_E_NOMEM;
  }
  c->ws_cap = cap;
  return MPC_OK;
}

// Bump allocator over the workspace for one call.
struct Carve {
  uint8_t* base;
  size_t off = 0;
  explicit Carve(uint8_t* b) : base(b) {}
  template <class T>
  T* take(size_t count) {
    T* p = (T*)(base + off);
    off += align_up(count * sizeof(T));
    return p;
  }
};

// Builder of one descriptor blob uploaded once per call.
struct Blob {
  std::vector<uint8_t> bytes;
  template <class T>
  size_t add(const T* src, size_t count) {
    size_t off = align_up(bytes.size(), 64);
    bytes.resize(off + align_up(count * sizeof(T), 64));
    if (count) std::memcpy(bytes.data() + off, src, count * sizeof(T));
    return off;
  }
};

// Uploads the blob; returns the device base address.  Eager calls use a ring
// of pinned slots (a slot is reused only after the call that used it has
// finished on the GPU); during capture the blob gets its own device buffer,
// filled before the graph exists, so the graph holds no copy node.
mpc_status upload(mpc_ctx* c, const Blob& b, uint8_t** dev) {
  const size_t n = std::max<size_t>(b.bytes.size(), 64);
  if (c->capturing) {
    void* d = nullptr;
    HIPCHK(hipMalloc(&d, n));
    c->capture_allocs.push_back(d);
    HIPCHK(hipMemcpyAsync(d, b.bytes.data(), b.bytes.size(), hipMemcpyHostToDevice, c->side));
    HIPCHK(hipStreamSynchronize(c->side));
    *dev = (uint8_t*)d;
    return MPC_OK;
  }
  UploadSlot& sl = c->slots[c->next_slot];
  c->cur_slot = c->next_slot;
  c->next_slot = (c->next_slot + 1) % kSlots;
  if (sl.pending) {
    HIPCHK(hipEventSynchronize(sl.done));
    sl.pending = false;
  }
  if (sl.cap < n) {
    if (sl.host) HIPCHK(hipHostFree(sl.host));
    if (sl.dev) HIPCHK(hipFree(sl.dev));
    sl.host = sl.dev = nullptr;
    sl.cap = 0;
    const size_t cap = align_up(n * 2, 1 << 16);
    HIPCHK(hipHostMalloc(&sl.host, cap, hipHostMallocDefault));
    HIPCHK(hipMalloc(&sl.dev, cap));
    sl.cap = cap;
  }
  std::memcpy(sl.host, b.bytes.data(), b.bytes.size());
  HIPCHK(hipMemcpyAsync(sl.dev, sl.host, b.bytes.size(), hipMemcpyHostToDevice, c->s[0]));
  *dev = (uint8_t*)sl.dev;
  return MPC_OK;
}

// The current upload slot may be reused once party 0's stream passes this
// point (every kernel reading it has been issued before).
mpc_status mark_slot(mpc_ctx* c) {
  if (c->cur_slot >= 0 && !c->capturing) {
    UploadSlot& sl = c->slots[c->cur_slot];
    HIPCHK(hipEventRecord(sl.done, c->s[0]));
    sl.pending = true;
  }
  c->cur_slot = -1;
  return MPC_OK;
}

// Marks the end of a call.
mpc_status end_call(mpc_ctx* c) { return mark_slot(c); }

bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

// Element counts above 2^46 (512 TiB of uint64) cannot be device buffers;
// refusing them keeps every size computed from a shape far from overflow.
constexpr i64 kMaxElems = (i64)1 << 46;
// Tile rows per raster group of the limb GEMM's schedule.
constexpr int kMaxGroupM = 64;
bool sched_ok(int variant, int group_m) {
  return variant >= 0 && variant < kLimbVariants && group_m >= 1 && group_m <= kMaxGroupM;
}

bool count_ok(i64 a, i64 b) { return a >= 0 && b >= 0 && (a == 0 || b <= kMaxElems / a); }

// M x K, K x N and M x N operands of a matrix product.
mpc_status check_mnk(i64 M, i64 N, i64 K) {
  if (M < 0 || N < 0 || K < 0) return MPC_E_SHAPE;
  return count_ok(M, K) && count_ok(K, N) && count_ok(M, N) ? MPC_OK : MPC_E_SHAPE;
}

mpc_status check_ptr(const void* p, size_t n) {
  if (n > (size_t)kMaxElems) return MPC_E_SHAPE;
  if (n == 0) return MPC_OK;
  if (!p || !aligned8(p)) return MPC_E_INVAL;
  return MPC_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || !na || !nb) return false;
  const uintptr_t a0 = (uintptr_t)a, a1 = a0 + na * 8, b0 = (uintptr_t)b, b1 = b0 + nb * 8;
  return a0 < b1 && b0 < a1;
}

// A batch's problems run concurrently: its outputs must be pairwise disjoint
// and must not overlap any input of the batch.  Sorted outputs, then one
// binary search per input.
struct Span {
  uintptr_t lo, hi;
};
void add_span(std::vector<Span>& v, const void* p, size_t n) {
  if (p && n) v.push_back(Span{(uintptr_t)p, (uintptr_t)p + n * 8});
}
mpc_status batch_disjoint(std::vector<Span> outs, const std::vector<Span>& ins) {
  std::sort(outs.begin(), outs.end(), [](const Span& a, const Span& b) { return a.lo < b.lo; });
  for (size_t i = 1; i < outs.size(); ++i)
    if (outs[i].lo < outs[i - 1].hi) return MPC_E_ALIAS;
  for (const Span& s : ins) {
    // the last output starting before s ends is the only one that can reach into s
    auto it = std::lower_bound(outs.begin(), outs.end(), s.hi,
                               [](const Span& o, uintptr_t v) { return o.lo < v; });
    if (it != outs.begin() && std::prev(it)->hi > s.lo) return MPC_E_ALIAS;
  }
  return MPC_OK;
}

mpc_status hip_status(hipError_t e) {
  if (e == hipSuccess) return MPC_OK;
  g_last_hip_error.store((int)e);
  return MPC_E_HIP;
}

mpc_status take_event(mpc_ctx* c, hipEvent_t* e) {
  if (!c->event_pool.empty()) {
    *e = c->event_pool.back();
    c->event_pool.pop_back();
    return MPC_OK;
  }
  HIPCHK(hipEventCreate(e));
  return MPC_OK;
}

// Brackets one GEMM launch with events when profiling (never inside a capture).
struct LaunchTimer {
  mpc_ctx* c;
  bool on;
  mpc_ctx::TimedLaunch rec{};
  LaunchTimer(mpc_ctx* ctx, int form, double macs) : c(ctx), on(ctx->profiling && !ctx->capturing) {
    rec.form = form;
    rec.ring_macs = macs;
  }
  mpc_status start() {
    if (!on) return MPC_OK;
    CHK(take_event(c, &rec.start));
    CHK(take_event(c, &rec.stop));
    HIPCHK(hipEventRecord(rec.start, c->s[0]));
    return MPC_OK;
  }
  mpc_status stop() {
    if (!on) return MPC_OK;
    HIPCHK(hipEventRecord(rec.stop, c->s[0]));
    c->timed.push_back(rec);
    return MPC_OK;
  }
};

OutView rowmajor_view(i64 N) { return OutView{N, std::max<i64>(N, 1), 0}; }

Epilogue make_ep(const u64* cadd, int csign, int trunc, u64* out, OutView v) {
  Epilogue e{};
  e.Cadd = cadd;
  e.csign = csign;
  e.trunc_bits = trunc;
  e.accumulate = 0;
  e.Out = out;
  e.view = v;
  return e;
}

// AUTO: the limb form for products of 2^22 ring MACs or more, when it can
// address their k segments (each kseg long; K is the total).
mpc_form resolve_form(mpc_form f, i64 M, i64 N, i64 K, i64 kseg) {
  if (f != MPC_FORM_AUTO) return f;
  if (kseg > kLimbMaxSegK) return MPC_FORM_PLAIN;
  const double work = (double)M * (double)N * (double)K;
  return work >= (double)(1 << 22) ? MPC_FORM_LIMB8 : MPC_FORM_PLAIN;
}

// The limb form asked for a k segment longer than it addresses.
mpc_status check_limb_k(mpc_form f, i64 kseg) {
  return f == MPC_FORM_LIMB8 && kseg > kLimbMaxSegK ? MPC_E_UNSUPPORTED : MPC_OK;
}

// ------------------------------------------------------------------ plain form
size_t packed_bytes(i64 rows, i64 K) {
  return (size_t)limb_rblocks(rows) * (size_t)limb_kblocks(K) * kLimbBlockBytes;
}

// Split-K plan of a plain launch: when the launch has fewer output tiles than
// compute units, long k ranges are cut into slices (at least kPlainMinSlice
// k each) so that about two workgroups per compute unit run; the slices'
// partial sums live in the context's split buffer.  Never grows that buffer
// during capture (the launch then runs unsplit).
constexpr i64 kPlainMinSlice = 32;

// Makes the split-K partial buffer at least `bytes` large; false when it
// would have to move while a graph is being captured or still refers to it
// (the caller then runs unsplit).
bool ensure_splitk(mpc_ctx* c, size_t bytes) {
  if (bytes <= c->splitk_cap) return true;
  if (c->capturing || c->live_graphs > 0) return false;
  if (sync_all(c) != MPC_OK) return false;
  if (c->splitk) (void)hipFree(c->splitk);
  c->splitk = nullptr;
  c->splitk_cap = 0;
  if (hipMalloc(&c->splitk, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  c->splitk_cap = bytes;
  return true;
}

mpc_status plan_splitk(mpc_ctx* c, std::vector<PlainProblem>& probs) {
  i64 tiles = 0;
  for (const PlainProblem& p : probs) tiles += plain_tiles(p.M, p.N);
  std::vector<int> ks(probs.size(), 1);
  size_t need = 0;
  if (tiles > 0 && tiles < c->num_cu) {
    const i64 want = (2 * (i64)c->num_cu + tiles - 1) / tiles;
    for (size_t q = 0; q < probs.size(); ++q) {
      const i64 Kt = probs[q].K0 + probs[q].K1;
      ks[q] = (int)std::max<i64>(1, std::min<i64>(want, Kt / kPlainMinSlice));
      if (ks[q] > 1) need += align_up((size_t)(ks[q] * probs[q].M * probs[q].N) * 8);
    }
  }
  if (need && !ensure_splitk(c, need)) {
    need = 0;
    std::fill(ks.begin(), ks.end(), 1);
  }
  size_t off = 0;
  for (size_t q = 0; q < probs.size(); ++q) {
    PlainProblem& p = probs[q];
    const i64 Kt = p.K0 + p.K1;
    if (ks[q] > 1) {
      const i64 per = (Kt + ks[q] - 1) / ks[q];
      p.kslice = (per + kPlainBK - 1) / kPlainBK * kPlainBK;
      p.ksplit = (int)((Kt + p.kslice - 1) / p.kslice);
      p.partial = (u64*)(c->splitk + off);
      off += align_up((size_t)(ks[q] * p.M * p.N) * 8);
    } else {
      p.ksplit = 1;
      p.kslice = std::max<i64>(Kt, 1);
      p.partial = nullptr;
    }
  }
  return MPC_OK;
}

// Split-K reductions of one call: their job table rides in the call's
// descriptor blob, and one launch reduces every split problem.
struct ReduceTable {
  size_t ojobs = 0, ostart = 0;
  int njobs = 0;
  i64 chunks = 0;
};
ReduceTable add_reduces(Blob& blob, const std::vector<ReduceJob>& jobs) {
  ReduceTable t;
  if (jobs.empty()) return t;
  std::vector<i64> cs(jobs.size() + 1, 0);
  for (size_t i = 0; i < jobs.size(); ++i) cs[i + 1] = cs[i] + (jobs[i].M * jobs[i].N + kReduceChunk - 1) / kReduceChunk;
  t.ojobs = blob.add(jobs.data(), jobs.size());
  t.ostart = blob.add(cs.data(), cs.size());
  t.njobs = (int)jobs.size();
  t.chunks = cs.back();
  return t;
}
mpc_status issue_reduces(mpc_ctx* c, hipStream_t st, const ReduceTable& t, const uint8_t* dev) {
  if (!t.njobs || !t.chunks) return MPC_OK;
  CHK(hip_status(launch_splitk_reduce_grouped(st, (const ReduceJob*)(dev + t.ojobs), (const i64*)(dev + t.ostart),
                                              t.njobs, t.chunks)));
  c->stats.launches++;
  return MPC_OK;
}

// One launch of the plain GEMM over `probs` (party 0's stream), plus one
// launch reducing every split problem.
mpc_status issue_plain(mpc_ctx* c, const std::vector<PlainProblem>& probs_in) {
  const size_t n = probs_in.size();
  if (!n) return MPC_OK;
  std::vector<PlainProblem> probs = probs_in;
  CHK(plan_splitk(c, probs));
  std::vector<int> tstart(n + 1, 0);
  double macs = 0;
  for (size_t q = 0; q < n; ++q) {
    tstart[q + 1] = tstart[q] + plain_tiles(probs[q].M, probs[q].N) * probs[q].ksplit;
    macs += (double)probs[q].M * (double)probs[q].N * (double)(probs[q].K0 + probs[q].K1);
  }
  std::vector<ReduceJob> reduces;
  for (const PlainProblem& p : probs)
    if (p.ksplit > 1) reduces.push_back(ReduceJob{p.partial, p.ksplit, p.M, p.N, p.ep});
  Blob blob;
  const size_t oprob = blob.add(probs.data(), n);
  const size_t otile = blob.add(tstart.data(), n + 1);
  const ReduceTable rt = add_reduces(blob, reduces);
  uint8_t* dev = nullptr;
  CHK(upload(c, blob, &dev));
  TileMap map{(int)n, (const int*)(dev + otile)};
  LaunchTimer tm(c, MPC_FORM_PLAIN, macs);
  CHK(tm.start());
  CHK(hip_status(launch_plain_gemm(c->s[0], (const PlainProblem*)(dev + oprob), map, tstart[n])));
  CHK(issue_reduces(c, c->s[0], rt, dev));
  CHK(tm.stop());
  c->stats.launches++;
  c->stats.gemm_problems += n;
  return MPC_OK;
}

PlainProblem plain_problem(i64 M, i64 N, i64 K0, i64 K1, const u64* A0, const u64* A0add, i64 lda0,
                           const u64* A1, i64 lda1, const u64* B0, const u64* B0add, i64 ldb0,
                           const u64* B1, i64 ldb1, const Epilogue& ep) {
  PlainProblem p{};
  p.M = M;
  p.N = N;
  p.K0 = K0;
  p.K1 = K1;
  p.A0 = A0;
  p.A0add = A0add;
  p.lda0 = lda0;
  p.A1 = A1;
  p.lda1 = lda1;
  p.B0 = B0;
  p.B0add = B0add;
  p.ldb0 = ldb0;
  p.B1 = B1;
  p.ldb1 = ldb1;
  p.ep = ep;
  return p;
}

// ------------------------------------------------------------------ fp64 limb form
// Workspace of one fp64-form ring GEMM of M x N over Kt concatenated k.
size_t fp64_ws(i64 M, i64 N, i64 Kt) {
  const i64 L = fp64_limbs(Kt);
  return align_up((size_t)(M * L * Kt) * 8) + align_up((size_t)(L * Kt * N) * 8) +
         align_up((size_t)(L * M * N) * 8);
}

// The vendor BLAS handle of the fp64 limb form, created on first use.  Its
// creation allocates device memory, so it cannot happen inside a graph
// capture: an fp64 call captured on a context that has never run one eagerly
// is refused (before it issues any work).
mpc_status fp64_ready(mpc_ctx* c) {
  if (c->blas) return MPC_OK;
  if (c->capturing) return MPC_E_UNSUPPORTED;
  if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
    c->blas = nullptr;
    return MPC_E_HIP;
  }
  return MPC_OK;
}

// C = [A0 | A1] @ [B0 ; B1] (mod 2^64) through fp64 limb planes and one vendor
// fp64 GEMM per diagonal, on party 0's stream; `cv` provides fp64_ws bytes.
mpc_status issue_fp64(mpc_ctx* c, Carve& cv, i64 M, i64 N, i64 K0, i64 K1, const u64* A0, i64 lda0,
                      const u64* A1, i64 lda1, const u64* B0, i64 ldb0, const u64* B1, i64 ldb1,
                      const Epilogue& ep) {
  const i64 Kt = K0 + K1;
  if (Kt >= kFp64MaxK) return MPC_E_UNSUPPORTED;
  CHK(fp64_ready(c));
  if (rocblas_set_stream(c->blas, c->s[0]) != rocblas_status_success) return MPC_E_HIP;
  const int L = fp64_limbs(Kt);
  double* LA = cv.take<double>((size_t)(M * L * Kt));
  double* RB = cv.take<double>((size_t)(L * Kt * N));
  double* X = cv.take<double>((size_t)(L * M * N));
  const hipStream_t st = c->s[0];
  if (Kt == 0) {
    // an empty sum: no diagonal enters the combine (no memory clearing, which
    // a graph capture should not record)
    CHK(hip_status(launch_fp64_combine(st, M, N, 0, X, ep)));
    c->stats.launches++;
    c->stats.gemm_problems++;
    return MPC_OK;
  }
  CHK(hip_status(launch_fp64_pack_left(st, M, K0, K1, A0, lda0, A1, lda1, L, LA)));
  CHK(hip_status(launch_fp64_pack_right(st, N, K0, K1, B0, ldb0, B1, ldb1, L, RB)));
  c->stats.launches += 2;
  // diagonal s: X_s = LA[:, 0:(s+1)Kt] @ RB[(L-1-s)Kt : L Kt, :]; row-major
  // products are issued as column-major X_s^T = RB_sub^T LA_sub^T
  const double one = 1.0, zero = 0.0;
  LaunchTimer tm(c, MPC_FORM_FP64LIMB, (double)M * (double)N * (double)Kt);
  CHK(tm.start());
  for (int sd = 0; sd < L; ++sd) {
    double* Xs = X + (size_t)sd * (size_t)(M * N);
    const rocblas_status bs = rocblas_dgemm(
        c->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)N, (rocblas_int)M,
        (rocblas_int)((sd + 1) * Kt), &one, RB + (size_t)(L - 1 - sd) * (size_t)Kt * (size_t)N,
        (rocblas_int)N, LA, (rocblas_int)(L * Kt), &zero, Xs, (rocblas_int)N);
    if (bs != rocblas_status_success) return MPC_E_HIP;
    c->stats.launches++;
  }
  CHK(tm.stop());
  CHK(hip_status(launch_fp64_combine(st, M, N, L, X, ep)));
  c->stats.launches++;
  c->stats.gemm_problems++;
  return MPC_OK;
}

// ------------------------------------------------------------------ limb form
// A pack job before its outputs are placed in the workspace.
struct JobSpec {
  int kind = kPackRow;
  int mode = kModeCopy;
  i64 rows = 0, K = 0, ld = 0;
  i64 cin = 0, len = 0, ksz = 1, stride = 1, lout = 1;
  const u64* in[kPackMaxIn] = {nullptr, nullptr, nullptr, nullptr};
  u64 key[2] = {0, 0};
  u64* share[2] = {nullptr, nullptr};
};

size_t job_bytes(const JobSpec& j) { return (size_t)pack_nout(j.mode) * align_up(packed_bytes(j.rows, j.K)); }

// Places a job's packed outputs in the workspace carve; with ws_outs >= 0
// only the first ws_outs of them (the caller points the rest elsewhere).
PackJob place_job(const JobSpec& j, Carve& cv, int ws_outs = -1) {
  PackJob p{};
  p.kind = j.kind;
  p.mode = j.mode;
  p.rows = j.rows;
  p.K = j.K;
  p.ld = j.ld;
  p.cin = j.cin;
  p.len = j.len;
  p.ksz = j.ksz;
  p.stride = j.stride;
  p.lout = j.lout;
  for (int i = 0; i < kPackMaxIn; ++i) p.in[i] = j.in[i];
  for (int i = 0; i < 2; ++i) {
    p.key[i] = j.key[i];
    p.share[i] = j.share[i];
  }
  p.rblocks = limb_rblocks(j.rows);
  p.rreal = (j.rows + 31) / 32;
  p.kblocks = limb_kblocks(j.K);
  const int nws = ws_outs < 0 ? pack_nout(j.mode) : ws_outs;
  for (int o = 0; o < kPackMaxOut; ++o)
    p.dst[o] = o < nws ? cv.take<uint8_t>(packed_bytes(j.rows, j.K)) : nullptr;
  return p;
}

// The offline-packed part of a matrix triple (the shares that enter the
// finish unchanged): a_1 as a left operand, b_0 and b_1 as right operands,
// each at its offset in one buffer.
size_t packed_triple_layout(i64 M, i64 N, i64 K, size_t off[3]) {
  off[0] = 0;
  off[1] = align_up(packed_bytes(M, K));
  off[2] = off[1] + align_up(packed_bytes(N, K));
  return off[2] + align_up(packed_bytes(N, K));
}

// Left operand MxK (row-major, leading dimension ld).
JobSpec left_job(i64 M, i64 K, i64 ld) {
  JobSpec j;
  j.kind = kPackRow;
  j.rows = M;
  j.K = K;
  j.ld = ld;
  return j;
}
// Right operand KxN (row-major, leading dimension ld).
JobSpec right_job(i64 K, i64 N, i64 ld) {
  JobSpec j;
  j.kind = kPackCol;
  j.rows = N;
  j.K = K;
  j.ld = ld;
  return j;
}
// Right operand im2col(x) of a [B][Cin][L] activation: K = Cin*k, N = B*Lout.
JobSpec im2col_job(const mpc_conv1d_shape& s, i64 lout) {
  JobSpec j;
  j.kind = kPackIm2col;
  j.rows = s.batch * lout;
  j.K = s.cin * s.ksize;
  j.cin = s.cin;
  j.len = s.length;
  j.ksz = s.ksize;
  j.stride = s.stride;
  j.lout = lout;
  return j;
}
void set_mode(JobSpec& j, int mode, std::initializer_list<const u64*> ins) {
  j.mode = mode;
  int n = 0;
  for (const u64* p : ins) j.in[n++] = p;
}
// Dealer operand drawn while it is packed: shares G(k0, e), G(k1, e) written
// to s0, s1, their sum packed.
void set_prg_sum2(JobSpec& j, u64 k0, u64 k1, u64* s0, u64* s1) {
  j.mode = kModePrgSum2;
  j.key[0] = k0;
  j.key[1] = k1;
  j.share[0] = s0;
  j.share[1] = s1;
}
// The fused open of a Beaver operand pair: (x, a) gives eps, g0 = a0 + eps and
// a1; (y, b) gives delta, b0 and b1.
void open_left(JobSpec& j, const u64* x0, const u64* x1, const u64* a0, const u64* a1) {
  set_mode(j, kModeOpenLeft, {x0, x1, a0, a1});
}
void open_right(JobSpec& j, const u64* y0, const u64* y1, const u64* b0, const u64* b1) {
  set_mode(j, kModeOpenRight, {y0, y1, b0, b1});
}

struct LimbReq {
  i64 M, N, K0, K1;
  const uint8_t *PA0, *PA1, *PB0, *PB1;
  Epilogue ep;
  bool own_sched;   // use `sched` instead of the call's schedule
  TileSched sched;
  int cls;          // tile class under the classes variants
};

// A rectangle of a product's output: rows [r0, r0 + m), columns [c0, c0 + n)
// in tile class cls.
struct Region {
  i64 r0, c0, m, n;
  int cls;
};

// The regions a request runs as (see issue_limb).  Every tile of a region
// reads only row and column blocks inside the product's packed operands,
// whose row and column counts are padded to multiples of 32 * kLimbRowPad:
// a strip's thin tiles span at most the padded extent of the rest (the
// 64-aligned part), and the corner's one 64x64 tile ends at most at the
// padded edge (checked below; otherwise the request is not split).
std::vector<Region> limb_regions(i64 M, i64 N, int cls, int variant, bool rowmajor) {
  const std::vector<Region> whole{Region{0, 0, M, N, cls}};
  if (!limb_per_class(variant) || cls != 0 || !rowmajor) return whole;
  const i64 rm = M % 64, rn = N % 64;
  const i64 m64 = (rm > 0 && rm <= 32) ? M - rm : M;
  const i64 n64 = (rn > 0 && rn <= 32) ? N - rn : N;
  if ((m64 == M && n64 == N) || m64 == 0 || n64 == 0) return whole;
  std::vector<Region> g{Region{0, 0, m64, n64, 0}};
  if (m64 < M) g.push_back(Region{m64, 0, M - m64, n64, 1});
  if (n64 < N) g.push_back(Region{0, n64, m64, N - n64, 2});
  if (m64 < M && n64 < N) g.push_back(Region{m64, n64, M - m64, N - n64, 0});
  const i64 rows = limb_rblocks(M) * 32, cols = limb_rblocks(N) * 32;
  i64 issued = 0;
  for (const Region& x : g) {
    int bm = 0, bn = 0;
    limb_class_shape(x.cls, &bm, &bn);
    const i64 tm = (x.m + bm - 1) / bm * bm, tn = (x.n + bn - 1) / bn * bn;
    if (x.r0 + tm > rows || x.c0 + tn > cols) return whole;
    issued += tm * tn;
  }
  // a strip beside at most 64 rows (columns) of interior issues as much as
  // the 64x64 tiles it replaces, in thinner tiles: keep the split only where
  // it issues less
  return issued < (M + 63) / 64 * 64 * ((N + 63) / 64 * 64) ? g : whole;
}
std::vector<Region> limb_regions(const LimbReq& r, const TileSched& ts) {
  return limb_regions(r.M, r.N, r.cls, ts.variant, r.ep.view.ld_q == 0 && r.ep.view.n_div >= r.N);
}

// One pack launch over all jobs, then one GEMM launch per K chunk (a problem
// whose concatenated K exceeds the int32-safe range continues in the next
// launch, adding into its output; truncation is applied by its last chunk).
// Descriptor tables go inside the kernels' arguments when every launch's are
// short (no upload), else in one upload for the call.  no_alloc: the caller
// cannot allocate, so no split-K (its partials and reduction table would need
// memory) and the tables must go inline; nothing is timed (timing events may
// be created on first use).
mpc_status issue_limb(mpc_ctx* c, const std::vector<PackJob>& jobs_in, const std::vector<LimbReq>& reqs,
                      TileSched sched, bool no_alloc = false) {
  // every entry point checks this before it issues any work
  for (const LimbReq& r : reqs)
    if (r.K0 > kLimbMaxSegK || r.K1 > kLimbMaxSegK) return MPC_E_UNSUPPORTED;
  hipStream_t st = c->s[0];
  // one pack launch per (kind, mode): the kernel is specialised on both
  std::vector<PackJob> jobs;
  std::vector<std::pair<int, int>> launch_km;
  std::vector<size_t> first_job;
  for (int kind : {kPackRow, kPackCol, kPackIm2col})
    for (int mode : {kModeCopy, kModeSum2, kModeOpenLeft, kModeOpenRight, kModePrgSum2, kModePrgSum2A, kModePrgSum2B,
                     kModeOpenLeft2, kModeOpenRight1}) {
      bool any = false;
      for (const PackJob& j : jobs_in) {
        if (j.kind != kind || j.mode != mode) continue;
        if (!any) {
          first_job.push_back(jobs.size());
          launch_km.push_back({kind, mode});
          any = true;
        }
        jobs.push_back(j);
      }
    }
  first_job.push_back(jobs.size());
  const size_t nj = jobs.size(), nreq = reqs.size();
  // per launch: prefix sums of its jobs' block counts
  std::vector<std::vector<i64>> bstarts(launch_km.size());
  for (size_t L = 0; L < launch_km.size(); ++L) {
    std::vector<i64>& bstart = bstarts[L];
    bstart.assign(1, 0);
    for (size_t i = first_job[L]; i < first_job[L + 1]; ++i)
      bstart.push_back(bstart.back() + jobs[i].rreal * jobs[i].kblocks);
  }

  // K pieces per request.  The int32 bound needs kbt / kLimbMaxKBlocks chunks,
  // run as consecutive launches that add into the output.  When the whole
  // launch has fewer tiles than compute units, k is instead cut into slices
  // (at least that many) that run side by side in one launch, each writing
  // its raw sum to a partial buffer; a reduction adds them and applies the
  // epilogue (split-K).
  std::vector<int> nchunks(nreq), nslices(nreq, 1);
  auto sched_of = [&](size_t q) { return reqs[q].own_sched ? reqs[q].sched : sched; };
  // Output regions of each request, each run as a problem of its own.  Under
  // a classes schedule a regular product whose last rows (columns) fill at
  // most half of a 64-row (64-column) tile runs those as a strip of 32x128
  // (128x32) tiles beside 64x64 tiles over the rest, and the corner they
  // share as one 64x64 tile: the padded work then follows the product's
  // edges at 32 instead of 64.  (Row-major outputs only: a region is a
  // pointer offset into the operands' packed row and column blocks and into
  // the output and triple share.)
  std::vector<std::vector<Region>> regions(nreq);
  // (not for a no-alloc call: its two problems must fit the kernel arguments)
  for (size_t q = 0; q < nreq; ++q)
    regions[q] = no_alloc ? std::vector<Region>{Region{0, 0, reqs[q].M, reqs[q].N, reqs[q].cls}}
                          : limb_regions(reqs[q], sched_of(q));
  auto tiles_of = [&](size_t q) {
    const TileSched t = sched_of(q);
    int n = 0;
    for (const Region& g : regions[q])
      n += limb_per_class(t.variant) ? limb_class_tiles(g.m, g.n, g.cls) : limb_tiles(g.m, g.n, t.variant);
    return n;
  };
  i64 tiles_all = 0;
  for (size_t q = 0; q < nreq; ++q) {
    const int kbt = (int)(limb_kblocks(reqs[q].K0) + limb_kblocks(reqs[q].K1));
    nchunks[q] = std::max(1, (kbt + kLimbMaxKBlocks - 1) / kLimbMaxKBlocks);
    tiles_all += tiles_of(q);
  }
  size_t part_bytes = 0;
  if (!no_alloc && tiles_all > 0 && tiles_all < c->num_cu) {
    const i64 want = (2 * (i64)c->num_cu + tiles_all - 1) / tiles_all;
    for (size_t q = 0; q < nreq; ++q) {
      const i64 steps = (limb_kblocks(reqs[q].K0) + limb_kblocks(reqs[q].K1)) / 2;
      const i64 sl = std::max<i64>(nchunks[q], std::min<i64>(want, steps / kLimbMinSliceSteps));
      if (sl > 1) {
        nslices[q] = (int)sl;
        part_bytes += align_up((size_t)(sl * reqs[q].M * reqs[q].N) * 8);
      }
    }
    if (part_bytes && !ensure_splitk(c, part_bytes)) {
      part_bytes = 0;
      std::fill(nslices.begin(), nslices.end(), 1);
    }
  }
  // GEMM launches: one per (K chunk, tile schedule), every launch of chunk ch
  // issued before any of chunk ch + 1 (which adds into chunk ch's outputs);
  // split-K slices all belong to chunk 0
  struct Launch {
    int chunk;
    TileSched sched;
    std::vector<LimbProblem> pieces;
    std::vector<int> tstarts{0};
    double macs = 0.0;
  };
  std::vector<Launch> launches;
  auto launch_of = [&](int chunk, const TileSched& ts) -> Launch& {
    for (Launch& l : launches)
      if (l.chunk == chunk && l.sched.variant == ts.variant && l.sched.group_m == ts.group_m &&
          l.sched.xcd_remap == ts.xcd_remap)
        return l;
    launches.push_back(Launch{chunk, ts, {}, {0}, 0.0});
    return launches.back();
  };
  std::vector<ReduceJob> reduces;
  size_t part_off = 0;
  for (size_t q = 0; q < nreq; ++q) {
    const LimbReq& r = reqs[q];
    const int kb0 = (int)limb_kblocks(r.K0), kb1 = (int)limb_kblocks(r.K1), kbt = kb0 + kb1;
    auto true_k = [&](i64 kb) {
      return kb <= kb0 ? std::min<i64>(kb * 32, r.K0) : r.K0 + std::min<i64>((kb - kb0) * 32, r.K1);
    };
    const TileSched ts = sched_of(q);
    auto piece = [&](int chunk, int kb_begin, int kb_end, const Epilogue& ep) -> mpc_status {
      // the GEMM steps over pairs of k-blocks inside one segment
      if ((kb0 | kb1 | kb_begin | kb_end) & 1) return MPC_E_INVAL;
      Launch& l = launch_of(chunk, ts);
      for (const Region& g : regions[q]) {
        LimbProblem p{};
        p.M = g.m;
        p.N = g.n;
        p.kb0 = kb0;
        p.kb1 = kb1;
        p.kb_begin = kb_begin;
        p.kb_end = kb_end;
        // a region starts at a whole 32-row (32-column) block: block (rb, kb)
        // of a segment sits at (rb * kblocks + kb) * 8 KiB
        const size_t ra = (size_t)(g.r0 / 32) * kLimbBlockBytes, cb = (size_t)(g.c0 / 32) * kLimbBlockBytes;
        p.PA0 = r.PA0 + ra * (size_t)kb0;
        p.PA1 = r.PA1 ? r.PA1 + ra * (size_t)kb1 : nullptr;
        p.PB0 = r.PB0 + cb * (size_t)kb0;
        p.PB1 = r.PB1 ? r.PB1 + cb * (size_t)kb1 : nullptr;
        p.mblocks = limb_rblocks(r.M) - g.r0 / 32;
        p.nblocks = limb_rblocks(r.N) - g.c0 / 32;
        p.ep = ep;
        const i64 eoff = g.r0 * ep.view.ld_m + g.c0;
        p.ep.Out = ep.Out + eoff;
        if (ep.Cadd) p.ep.Cadd = ep.Cadd + eoff;
        p.cls = g.cls;
        l.pieces.push_back(p);
        l.tstarts.push_back(l.tstarts.back() +
                            (limb_per_class(ts.variant) ? limb_class_tiles(g.m, g.n, g.cls)
                                                        : limb_tiles(g.m, g.n, ts.variant)));
      }
      l.macs += (double)r.M * (double)r.N * (double)(true_k(kb_end) - true_k(kb_begin));
      return MPC_OK;
    };
    if (nslices[q] > 1) {
      const int ks = nslices[q];
      const i64 steps = kbt / 2;
      u64* part = (u64*)(c->splitk + part_off);
      part_off += align_up((size_t)(ks * r.M * r.N) * 8);
      for (int sl = 0; sl < ks; ++sl) {
        const int b0 = (int)(2 * (steps * sl / ks)), b1 = (int)(2 * (steps * (sl + 1) / ks));
        CHK(piece(0, b0, b1, make_ep(nullptr, +1, 0, part + (size_t)sl * (size_t)(r.M * r.N), rowmajor_view(r.N))));
      }
      reduces.push_back(ReduceJob{part, ks, r.M, r.N, r.ep});
    } else {
      for (int ch = 0; ch < nchunks[q]; ++ch) {
        Epilogue ep = r.ep;
        if (ch > 0) {
          ep.accumulate = 1;
          ep.Cadd = nullptr;
        }
        if (ch + 1 < nchunks[q]) ep.trunc_bits = 0;
        CHK(piece(ch, std::min(kbt, ch * kLimbMaxKBlocks), std::min(kbt, (ch + 1) * kLimbMaxKBlocks), ep));
      }
    }
  }
  std::stable_sort(launches.begin(), launches.end(),
                   [](const Launch& a, const Launch& b) { return a.chunk < b.chunk; });
  const size_t nlaunch = launches.size();
  bool inl = reduces.empty();
  for (size_t L = 0; L < launch_km.size(); ++L)
    if (first_job[L + 1] - first_job[L] > (size_t)kInlineJobs) inl = false;
  for (const Launch& l : launches)
    if (l.pieces.size() > (size_t)kInlineProbs) inl = false;
  // with split-K off, a no-alloc call has one job per operand side and two
  // problems per launch
  if (no_alloc && !inl) return MPC_E_UNSUPPORTED;
  Blob blob;
  std::vector<size_t> obstart(launch_km.size()), oprob(nlaunch), otile(nlaunch);
  size_t ojobs = 0;
  ReduceTable rt{};
  uint8_t* dev = nullptr;
  if (!inl) {
    for (size_t L = 0; L < launch_km.size(); ++L) obstart[L] = blob.add(bstarts[L].data(), bstarts[L].size());
    ojobs = blob.add(jobs.data(), nj);
    for (size_t L = 0; L < nlaunch; ++L) {
      oprob[L] = blob.add(launches[L].pieces.data(), launches[L].pieces.size());
      otile[L] = blob.add(launches[L].tstarts.data(), launches[L].tstarts.size());
    }
    rt = add_reduces(blob, reduces);
    CHK(upload(c, blob, &dev));
  }
  for (size_t L = 0; L < launch_km.size(); ++L) {
    const int njl = (int)(first_job[L + 1] - first_job[L]);
    PackTables t{};
    t.njobs = njl;
    if (inl) {
      for (int i = 0; i < njl; ++i) t.ijobs[i] = jobs[first_job[L] + i];
      for (int i = 0; i <= njl; ++i) t.ibstart[i] = bstarts[L][i];
    } else {
      t.jobs = (const PackJob*)(dev + ojobs) + first_job[L];
      t.block_start = (const i64*)(dev + obstart[L]);
    }
    CHK(hip_status(launch_pack(st, t, bstarts[L].back(), launch_km[L].first, launch_km[L].second)));
    c->stats.launches++;
  }
  for (size_t L = 0; L < nlaunch; ++L) {
    const Launch& l = launches[L];
    if (l.pieces.empty()) continue;
    GemmTables t{};
    t.sched = l.sched;
    t.map.nprob = (int)l.pieces.size();
    t.queue = c->queue;
    t.persist_grid = limb_persist_grid(l.tstarts.back(), c->num_cu);
    if (inl) {
      for (size_t i = 0; i < l.pieces.size(); ++i) t.iprobs[i] = l.pieces[i];
      for (size_t i = 0; i < l.tstarts.size(); ++i) t.itile_start[i] = l.tstarts[i];
    } else {
      t.probs = (const LimbProblem*)(dev + oprob[L]);
      t.map.tile_start = (const int*)(dev + otile[L]);
    }
    LaunchTimer tm(c, MPC_FORM_LIMB8, l.macs);
    if (no_alloc) tm.on = false;
    CHK(tm.start());
    CHK(hip_status(launch_limb_gemm(st, t, l.tstarts.back())));
    CHK(tm.stop());
    c->stats.launches++;
  }
  if (!inl) CHK(issue_reduces(c, st, rt, dev));
  c->stats.gemm_problems += nreq;
  return MPC_OK;
}

LimbReq limb_req(i64 M, i64 N, i64 K0, i64 K1, const uint8_t* PA0, const uint8_t* PA1,
                 const uint8_t* PB0, const uint8_t* PB1, const Epilogue& ep) {
  return LimbReq{M, N, K0, K1, PA0, PA1, PB0, PB1, ep, false, TileSched{}, 0};
}

mpc_status check_trunc(int bits) { return (bits < 0 || bits > 63) ? MPC_E_INVAL : MPC_OK; }
mpc_status check_form(mpc_form f) {
  return (f == MPC_FORM_PLAIN || f == MPC_FORM_LIMB8 || f == MPC_FORM_AUTO || f == MPC_FORM_FP64LIMB)
             ? MPC_OK
             : MPC_E_INVAL;
}


i64 conv_lout(const mpc_conv1d_shape& s) {
  return s.length < s.ksize ? 0 : (s.length - s.ksize) / s.stride + 1;
}

mpc_status check_conv(const mpc_conv1d_shape* s) {
  if (!s) return MPC_E_INVAL;
  if (s->batch < 0 || s->cin < 0 || s->length < 0 || s->cout < 0 || s->ksize <= 0 || s->stride <= 0)
    return MPC_E_SHAPE;
  // activation, weight and output tensors, and the lowered product's k x n
  const i64 lout = conv_lout(*s);
  const bool ok = count_ok(s->batch, s->cin) && count_ok(s->batch * s->cin, s->length) &&
                  count_ok(s->cout, s->cin) && count_ok(s->cout * s->cin, s->ksize) && count_ok(s->batch, lout) &&
                  count_ok(s->cout, s->batch * lout) && count_ok(s->cin, s->ksize) &&
                  count_ok(s->cin * s->ksize, s->batch * lout);
  return ok ? MPC_OK : MPC_E_SHAPE;
}

}  // namespace

// ====================================================================== API
extern "C" {

const char* mpc_status_str(mpc_status s) {
  switch (s) {
    case MPC_OK: return "ok";
    case MPC_E_INVAL: return "invalid argument";
    case MPC_E_SHAPE: return "invalid shape";
    case MPC_E_ALIAS: return "output overlaps an input";
    case MPC_E_NOMEM: return "workspace allocation failed";
    case MPC_E_HIP: return "HIP runtime error";
    case MPC_E_UNSUPPORTED: return "unsupported";
    case MPC_E_RANGE: return "value outside the fixed-point range";
  }
  return "unknown status";
}

int mpc_last_hip_error(void) { return g_last_hip_error.load(); }

mpc_status mpc_encode(const double* x, size_t n, int frac_bits, int64_t* out) {
  if (n && (!x || !out)) return MPC_E_INVAL;
  if (frac_bits < 0 || frac_bits > 62) return MPC_E_INVAL;
  const double scale = std::ldexp(1.0, frac_bits);
  for (size_t i = 0; i < n; ++i) {
    const double r = std::nearbyint(x[i] * scale);  // ties to even in the default mode
    if (!(r >= -9223372036854775808.0 && r < 9223372036854775808.0)) return MPC_E_RANGE;
    out[i] = (int64_t)r;
  }
  return MPC_OK;
}

mpc_status mpc_decode(const int64_t* v, size_t n, int frac_bits, double* out) {
  if (n && (!v || !out)) return MPC_E_INVAL;
  if (frac_bits < 0 || frac_bits > 62) return MPC_E_INVAL;
  const double inv = std::ldexp(1.0, -frac_bits);
  for (size_t i = 0; i < n; ++i) out[i] = (double)v[i] * inv;
  return MPC_OK;
}

mpc_status mpc_ctx_create(int device, void* stream0, void* stream1, uint64_t seed, mpc_ctx** out) {
  if (!out) return MPC_E_INVAL;
  *out = nullptr;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return MPC_E_INVAL;
  mpc_ctx* c = new (std::nothrow) mpc_ctx();
  if (!c) return MPC_E_NOMEM;
  c->device = device;
  c->seed = seed;
  auto fail = [&](hipError_t e) {
    g_last_hip_error.store((int)e);
    mpc_ctx_destroy(c);
    return MPC_E_HIP;
  };
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return fail(e);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return fail(e);
  c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  // party 0: the given stream (NULL is the device's null stream); party 1: the
  // given stream, or a stream the library creates and owns when NULL
  c->s[0] = (hipStream_t)stream0;
  if (stream1) {
    c->s[1] = (hipStream_t)stream1;
  } else {
    e = hipStreamCreateWithFlags(&c->s[1], hipStreamNonBlocking);
    if (e != hipSuccess) return fail(e);
    c->own[1] = true;
  }
  for (int p = 0; p < 2; ++p) {
    e = hipEventCreateWithFlags(&c->ev[p], hipEventDisableTiming);
    if (e != hipSuccess) return fail(e);
  }
  e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  if (e != hipSuccess) return fail(e);
  for (int i = 0; i < kSlots; ++i) {
    e = hipEventCreateWithFlags(&c->slots[i].done, hipEventDisableTiming);
    if (e != hipSuccess) return fail(e);
  }
  e = hipMalloc((void**)&c->queue, kLimbQueueWords * sizeof(unsigned));
  if (e != hipSuccess) return fail(e);
  {
    // a copy from pageable host memory has completed when it returns, so the
    // zeros are in place before any stream's first launch
    const unsigned zeros[kLimbQueueWords] = {};
    e = hipMemcpy(c->queue, zeros, sizeof(zeros), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(e);
  }
  // the device is current: find its no-alloc workspace (a failure only
  // disables mpc_beaver_matmul_noalloc)
  c->scratch = (uint8_t*)scratch_address(device);
  *out = c;
  return MPC_OK;
}

mpc_status mpc_ctx_destroy(mpc_ctx* c) {
  if (!c) return MPC_OK;
  // its graphs hold the context's address and buffers
  if (c->live_graphs > 0) return MPC_E_INVAL;
  (void)hipSetDevice(c->device);
  for (int p = 0; p < 2; ++p)
    if (c->s[p]) (void)hipStreamSynchronize(c->s[p]);
  if (c->side) (void)hipStreamSynchronize(c->side);
  for (int i = 0; i < kSlots; ++i) {
    UploadSlot& sl = c->slots[i];
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.dev) (void)hipFree(sl.dev);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  for (void* p : c->capture_allocs) (void)hipFree(p);
  if (c->queue) (void)hipFree(c->queue);
  for (auto& t : c->timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->blas) (void)rocblas_destroy_handle(c->blas);
  if (c->splitk) (void)hipFree(c->splitk);
  if (c->ws) (void)hipFree(c->ws);
  for (int p = 0; p < 2; ++p) {
    if (c->ev[p]) (void)hipEventDestroy(c->ev[p]);
    if (c->own[p] && c->s[p]) (void)hipStreamDestroy(c->s[p]);
  }
  if (c->side) (void)hipStreamDestroy(c->side);
  delete c;
  return MPC_OK;
}

mpc_status mpc_sync(mpc_ctx* c) {
  if (!c) return MPC_E_INVAL;
  CHK(set_device(c));
  return sync_all(c);
}

mpc_status mpc_ctx_stats(const mpc_ctx* c, mpc_stats* out) {
  if (!c || !out) return MPC_E_INVAL;
  *out = c->stats;
  return MPC_OK;
}

mpc_status mpc_reserve(mpc_ctx* c, size_t bytes) {
  if (!c) return MPC_E_INVAL;
  CHK(set_device(c));
  return ensure_ws(c, bytes);
}

// ------------------------------------------------------------------ sharing
mpc_status mpc_share(mpc_ctx* c, const uint64_t* x, size_t n, int src, uint64_t tag, uint64_t* s0,
                     uint64_t* s1) {
  if (!c || (src != 0 && src != 1)) return MPC_E_INVAL;
  CHK(check_ptr(x, n));
  CHK(check_ptr(s0, n));
  CHK(check_ptr(s1, n));
  if (overlap(s0, n, x, n) || overlap(s1, n, x, n) || overlap(s0, n, s1, n)) return MPC_E_ALIAS;
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_share(c->s[0], x, n, src, stream_key(c->seed, tag, kSlotShare), s0, s1)));
  c->stats.launches++;
  return end_call(c);
}

mpc_status mpc_reveal(mpc_ctx* c, const uint64_t* s0, const uint64_t* s1, size_t n, uint64_t* out) {
  if (!c) return MPC_E_INVAL;
  CHK(check_ptr(s0, n));
  CHK(check_ptr(s1, n));
  CHK(check_ptr(out, n));
  // in place (out is s0 or s1) is element-wise safe; any other overlap is not
  if ((out != s0 && overlap(out, n, s0, n)) || (out != s1 && overlap(out, n, s1, n))) return MPC_E_ALIAS;
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_reveal(c->s[0], s0, s1, n, out)));
  c->stats.launches++;
  c->stats.opens++;  // each party sends its share: one round
  c->stats.open_bytes_per_party += 8 * (uint64_t)n;
  return end_call(c);
}

mpc_status mpc_truncate(mpc_ctx* c, uint64_t* s0, uint64_t* s1, size_t n, int bits) {
  if (!c) return MPC_E_INVAL;
  CHK(check_trunc(bits));
  CHK(check_ptr(s0, n));
  CHK(check_ptr(s1, n));
  if (overlap(s0, n, s1, n)) return MPC_E_ALIAS;
  if (!n || !bits) return MPC_OK;
  CHK(set_device(c));
  // each party truncates its own share on its own stream: no communication
  CHK(fork(c));
  CHK(hip_status(launch_truncate(c->s[0], s0, n, bits)));
  CHK(hip_status(launch_truncate(c->s[1], s1, n, bits)));
  CHK(join(c));
  c->stats.launches += 2;
  c->stats.truncations++;
  return end_call(c);
}

// ------------------------------------------------------------------ dealer
mpc_status mpc_dealer_triples(mpc_ctx* c, mpc_triple_kind kind, uint64_t dseed, uint64_t tag,
                              const int64_t* dims, const mpc_triple* t) {
  if (!c || !dims || !t) return MPC_E_INVAL;
  u64 key[6];
  for (int sl = 0; sl < 6; ++sl) key[sl] = stream_key(dseed, tag, (u64)sl);
  CHK(set_device(c));
  hipStream_t st = c->s[0];
  if (kind == MPC_TRIPLE_MUL || kind == MPC_TRIPLE_SQUARE) {
    if (dims[0] < 0) return MPC_E_SHAPE;
    const size_t n = (size_t)dims[0];
    const bool sq = kind == MPC_TRIPLE_SQUARE;
    uint64_t* bufs[6] = {t->a0, t->a1, t->b0, t->b1, t->c0, t->c1};
    const int nb = sq ? 4 : 6;
    for (int i = 0; i < nb; ++i) {
      CHK(check_ptr(bufs[i], n));
      for (int j = 0; j < i; ++j)
        if (overlap(bufs[i], n, bufs[j], n)) return MPC_E_ALIAS;
    }
    if (!n) return MPC_OK;
    if (sq) CHK(hip_status(launch_dealer_square(st, key, n, t->a0, t->a1, t->b0, t->b1)));
    else CHK(hip_status(launch_dealer_mul(st, key, n, t->a0, t->a1, t->b0, t->b1, t->c0, t->c1)));
    c->stats.launches++;
    return end_call(c);
  }
  if (kind != MPC_TRIPLE_MATMUL && kind != MPC_TRIPLE_CONV1D) return MPC_E_INVAL;

  // c = f(a0 + a1, b0 + b1), c1 = c - c0, as one ring GEMM whose operands are
  // formed while they are loaded (plain) or packed (limb).
  size_t na, nb, nc;
  i64 M, N, K, lout = 0;
  mpc_conv1d_shape cs{};
  OutView view;
  if (kind == MPC_TRIPLE_MATMUL) {
    M = dims[0];
    N = dims[1];
    K = dims[2];
    CHK(check_mnk(M, N, K));
    na = (size_t)(M * K);
    nb = (size_t)(K * N);
    nc = (size_t)(M * N);
    view = rowmajor_view(N);
  } else {
    cs = {dims[0], dims[1], dims[2], dims[3], dims[4], dims[5]};
    CHK(check_conv(&cs));
    lout = conv_lout(cs);
    na = (size_t)(cs.batch * cs.cin * cs.length);
    nb = (size_t)(cs.cout * cs.cin * cs.ksize);
    nc = (size_t)(cs.batch * cs.cout * lout);
    // transposed orientation: c[b][o][l] = (Wm(b) @ im2col(a))[o][b*Lout + l]
    M = cs.cout;
    N = cs.batch * lout;
    K = cs.cin * cs.ksize;
    view = OutView{lout, std::max<i64>(lout, 1), cs.cout * lout};
  }
  CHK(check_ptr(t->a0, na));
  CHK(check_ptr(t->a1, na));
  CHK(check_ptr(t->b0, nb));
  CHK(check_ptr(t->b1, nb));
  CHK(check_ptr(t->c0, nc));
  CHK(check_ptr(t->c1, nc));
  const void* bufs[6] = {t->a0, t->a1, t->b0, t->b1, t->c0, t->c1};
  const size_t ns[6] = {na, na, nb, nb, nc, nc};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < i; ++j)
      if (overlap(bufs[i], ns[i], bufs[j], ns[j])) return MPC_E_ALIAS;

  const mpc_form form = resolve_form(MPC_FORM_AUTO, M, N, K, K);
  const Epilogue ep = make_ep(t->c0, -1, 0, t->c1, view);
  // the left factor is a (matmul) or the weight b (conv); the right one b or im2col(a)
  const u64 *L0 = kind == MPC_TRIPLE_MATMUL ? t->a0 : t->b0, *L1 = kind == MPC_TRIPLE_MATMUL ? t->a1 : t->b1;
  const u64 *R0 = kind == MPC_TRIPLE_MATMUL ? t->b0 : t->a0, *R1 = kind == MPC_TRIPLE_MATMUL ? t->b1 : t->a1;
  JobSpec jl = left_job(M, K, K), jr = kind == MPC_TRIPLE_MATMUL ? right_job(K, N, N) : im2col_job(cs, lout);
  set_mode(jl, kModeSum2, {L0, L1});
  set_mode(jr, kModeSum2, {R0, R1});
  // In the limb form a matrix operand's shares are drawn inside its pack
  // (each element is packed exactly once), so they are written once and never
  // read back; an im2col operand (overlapping windows, possibly uncovered
  // tail elements) and the plain form take the shares from PRG fills.
  const bool limb = form == MPC_FORM_LIMB8 && nc > 0;
  const bool a_left = kind == MPC_TRIPLE_MATMUL;  // which triple factor is the left operand
  u64* Ls[2] = {a_left ? t->a0 : t->b0, a_left ? t->a1 : t->b1};
  u64* Rs[2] = {a_left ? t->b0 : t->a0, a_left ? t->b1 : t->a1};
  const int Lslot = a_left ? kSlotA0 : kSlotB0, Rslot = a_left ? kSlotB0 : kSlotA0;
  const bool fuse_r = limb && kind == MPC_TRIPLE_MATMUL;
  if (limb) set_prg_sum2(jl, key[Lslot], key[Lslot + 1], Ls[0], Ls[1]);
  if (fuse_r) set_prg_sum2(jr, key[Rslot], key[Rslot + 1], Rs[0], Rs[1]);
  size_t need = kAlign;
  if (form == MPC_FORM_LIMB8) need += job_bytes(jl) + job_bytes(jr);
  else if (kind == MPC_TRIPLE_CONV1D) need += align_up((size_t)(K * N) * 8);
  CHK(ensure_ws(c, need));
  const size_t nl = a_left ? na : nb, nr = a_left ? nb : na;
  if (!limb) {
    CHK(hip_status(launch_prg_fill(st, key[Lslot], Ls[0], nl)));
    CHK(hip_status(launch_prg_fill(st, key[Lslot + 1], Ls[1], nl)));
    c->stats.launches += 2;
  }
  if (!fuse_r) {
    CHK(hip_status(launch_prg_fill(st, key[Rslot], Rs[0], nr)));
    CHK(hip_status(launch_prg_fill(st, key[Rslot + 1], Rs[1], nr)));
    c->stats.launches += 2;
  }
  CHK(hip_status(launch_prg_fill(st, key[kSlotC0], t->c0, nc)));
  c->stats.launches += 1;
  if (nc) {
    Carve cv(c->ws);
    if (form == MPC_FORM_LIMB8) {
      std::vector<PackJob> jobs{place_job(jl, cv), place_job(jr, cv)};
      CHK(issue_limb(c, jobs, {limb_req(M, N, K, 0, jobs[0].dst[0], nullptr, jobs[1].dst[0], nullptr, ep)}, c->sched_default));
    } else if (kind == MPC_TRIPLE_MATMUL) {
      CHK(issue_plain(c, {plain_problem(M, N, K, 0, L0, L1, K, nullptr, 0, R0, R1, N, nullptr, 0, ep)}));
    } else {
      u64* col = cv.take<u64>((size_t)(K * N));
      CHK(hip_status(launch_im2col(st, R0, R1, cs.batch, cs.cin, cs.length, cs.ksize, cs.stride, lout, col)));
      c->stats.launches++;
      CHK(issue_plain(c, {plain_problem(M, N, K, 0, L0, L1, K, nullptr, 0, col, nullptr, N, nullptr, 0, ep)}));
    }
  }
  return end_call(c);
}

// ------------------------------------------------------------------ Beaver
mpc_status mpc_beaver_mul(mpc_ctx* c, size_t n, const uint64_t* x0, const uint64_t* x1,
                          const uint64_t* y0, const uint64_t* y1, const mpc_triple* t, int trunc_bits,
                          uint64_t* z0, uint64_t* z1) {
  if (!c || !t) return MPC_E_INVAL;
  CHK(check_trunc(trunc_bits));
  const bool sq = (y0 == nullptr && y1 == nullptr);
  if (!sq && (y0 == nullptr || y1 == nullptr)) return MPC_E_INVAL;
  const void* ins[10] = {x0, x1, y0, y1, t->a0, t->a1, t->b0, t->b1, t->c0, t->c1};
  const int nin = sq ? 8 : 10;
  for (int i = 0; i < nin; ++i) {
    if (sq && (i == 2 || i == 3)) continue;
    CHK(check_ptr(ins[i], n));
  }
  CHK(check_ptr(z0, n));
  CHK(check_ptr(z1, n));
  if (overlap(z0, n, z1, n)) return MPC_E_ALIAS;
  for (int i = 0; i < nin; ++i)
    if (overlap(z0, n, ins[i], n) || overlap(z1, n, ins[i], n)) return MPC_E_ALIAS;
  if (!n) return MPC_OK;
  CHK(set_device(c));
  if (sq)
    CHK(hip_status(launch_beaver_square(c->s[0], n, x0, x1, t->a0, t->a1, t->b0, t->b1, trunc_bits, z0, z1)));
  else
    CHK(hip_status(launch_beaver_mul(c->s[0], n, x0, x1, y0, y1, t->a0, t->a1, t->b0, t->b1, t->c0, t->c1,
                                     trunc_bits, z0, z1)));
  c->stats.launches++;
  c->stats.opens++;
  c->stats.open_bytes_per_party += (sq ? 1 : 2) * 8 * (uint64_t)n;
  if (trunc_bits) c->stats.truncations++;
  return end_call(c);
}

namespace {

// FNV-1a hash of a list of matmul shapes (in the order the GEMM issues them).
uint64_t shapes_key(const std::vector<std::array<i64, 3>>& shapes) {
  uint64_t h = 1469598103934665603ULL;
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xff;
      h *= 1099511628211ULL;
    }
  };
  mix(shapes.size());
  for (const auto& s : shapes)
    for (i64 v : s) mix((uint64_t)v);
  return h;
}

int bucket_of(i64 M, i64 N) {
  auto padded = [&](i64 bm, i64 bn) { return (double)((M + bm - 1) / bm * bm) * (double)((N + bn - 1) / bn * bn); };
  const double reg = padded(64, 64), tm = padded(32, 128), tn = padded(128, 32);
  if (M <= 32 && tm <= 0.9 * reg && tm <= tn) return kBucketThinM;
  if (N <= 32 && tn <= 0.9 * reg) return kBucketThinN;
  return kBucketRegular;
}

// A problem's schedule and, under the classes variants, its tile class.
struct ProbSched {
  TileSched s;
  int cls;
};

// The schedule of every problem of a matmul shape list.  Tuned: its class's
// schedule for this list.  Untuned: the default schedule (a classes schedule
// with each problem's own class), unless some product is thin and no default
// was set: then every problem runs in the one classes launch with its own
// class.
std::vector<ProbSched> scheds_for(const mpc_ctx* c, const std::vector<std::array<i64, 3>>& shapes) {
  std::vector<ProbSched> out;
  auto it = c->tuned.find(shapes_key(shapes));
  bool thin = false;
  for (const auto& sh : shapes) thin = thin || bucket_of(sh[0], sh[1]) != kBucketRegular;
  const TileSched d = c->sched_default;
  for (const auto& sh : shapes) {
    const int b = bucket_of(sh[0], sh[1]);
    if (it != c->tuned.end()) out.push_back(ProbSched{it->second.s[b], b});
    else if (c->class_tiles && thin) out.push_back(ProbSched{TileSched{kLimbClasses, d.group_m, d.xcd_remap}, b});
    else out.push_back(ProbSched{d, limb_per_class(d.variant) ? b : 0});
  }
  return out;
}

}  // namespace

namespace {

// One Beaver matmul of the call (a grouped call holds many).  `packed`: the
// triple's offline-packed a_1, b_0, b_1 (packed_triple_layout), or null.
struct MatmulPlan {
  i64 M, N, K;
  const u64 *x0, *x1, *y0, *y1;
  mpc_triple t;
  u64 *z0, *z1;
  const uint8_t* packed = nullptr;
};

mpc_status validate_matmul(const MatmulPlan& m) {
  CHK(check_mnk(m.M, m.N, m.K));
  const size_t na = (size_t)(m.M * m.K), nb = (size_t)(m.K * m.N), nc = (size_t)(m.M * m.N);
  const void* in[10] = {m.x0, m.x1, m.y0, m.y1, m.t.a0, m.t.a1, m.t.b0, m.t.b1, m.t.c0, m.t.c1};
  const size_t ns[10] = {na, na, nb, nb, na, na, nb, nb, nc, nc};
  for (int i = 0; i < 10; ++i) CHK(check_ptr(in[i], ns[i]));
  CHK(check_ptr(m.z0, nc));
  CHK(check_ptr(m.z1, nc));
  if (overlap(m.z0, nc, m.z1, nc)) return MPC_E_ALIAS;
  for (int i = 0; i < 10; ++i)
    if (overlap(m.z0, nc, in[i], ns[i]) || overlap(m.z1, nc, in[i], ns[i])) return MPC_E_ALIAS;
  return MPC_OK;
}

// Open step of the plain form: one launch over all jobs (device job table).
mpc_status issue_opens(mpc_ctx* c, const std::vector<OpenJob>& opens) {
  if (opens.empty()) return MPC_OK;
  std::vector<i64> cs(opens.size() + 1, 0);
  for (size_t i = 0; i < opens.size(); ++i) cs[i + 1] = cs[i] + (opens[i].n + kOpenChunk - 1) / kOpenChunk;
  Blob blob;
  const size_t ojobs = blob.add(opens.data(), opens.size());
  const size_t ostart = blob.add(cs.data(), cs.size());
  uint8_t* dev = nullptr;
  CHK(upload(c, blob, &dev));
  // this slot is read only by the open launch
  if (c->cur_slot >= 0 && !c->capturing) {
    const int slot = c->cur_slot;
    CHK(hip_status(launch_open(c->s[0], (const OpenJob*)(dev + ojobs), (const i64*)(dev + ostart),
                               (int)opens.size(), cs.back())));
    HIPCHK(hipEventRecord(c->slots[slot].done, c->s[0]));
    c->slots[slot].pending = true;
  } else {
    CHK(hip_status(launch_open(c->s[0], (const OpenJob*)(dev + ojobs), (const i64*)(dev + ostart),
                               (int)opens.size(), cs.back())));
  }
  c->stats.launches++;
  return MPC_OK;
}

// Workspace of one Beaver matmul in a form.
size_t matmul_ws(const MatmulPlan& m, mpc_form form) {
  if (form == MPC_FORM_LIMB8 && m.packed)  // eps, g0 and delta only
    return 2 * align_up(packed_bytes(m.M, m.K)) + align_up(packed_bytes(m.N, m.K));
  if (form == MPC_FORM_LIMB8)
    return 3 * align_up(packed_bytes(m.M, m.K)) + 3 * align_up(packed_bytes(m.N, m.K));
  return 2 * align_up((size_t)(m.M * m.K) * 8) + align_up((size_t)(m.K * m.N) * 8);
}

// Plain-form opens, then each party's finish z_p = c_p + [eps | g_p] @ [b_p ; delta]
// in the fp64 limb form, one party after the other through one shared
// fp64 workspace (all on party 0's stream).
mpc_status run_matmuls_fp64(mpc_ctx* c, const std::vector<MatmulPlan>& plans, int trunc) {
  size_t need = kAlign, fp = 0;
  for (const MatmulPlan& m : plans) {
    if (2 * m.K >= kFp64MaxK) return MPC_E_UNSUPPORTED;
    need += matmul_ws(m, MPC_FORM_PLAIN);
    fp = std::max(fp, fp64_ws(m.M, m.N, 2 * m.K));
  }
  CHK(fp64_ready(c));
  CHK(ensure_ws(c, need + fp));
  Carve cv(c->ws);
  std::vector<OpenJob> opens;
  struct Opened { u64 *eps, *g, *del; };
  std::vector<Opened> op;
  for (const MatmulPlan& m : plans) {
    u64* eps = cv.take<u64>((size_t)(m.M * m.K));
    u64* g = cv.take<u64>((size_t)(m.M * m.K));
    u64* del = cv.take<u64>((size_t)(m.K * m.N));
    opens.push_back(OpenJob{kOpenLeft, m.M * m.K, m.x0, m.x1, m.t.a0, m.t.a1, eps, g});
    opens.push_back(OpenJob{kOpenRight, m.K * m.N, m.y0, m.y1, m.t.b0, m.t.b1, del, nullptr});
    op.push_back(Opened{eps, g, del});
  }
  CHK(issue_opens(c, opens));
  for (size_t q = 0; q < plans.size(); ++q) {
    const MatmulPlan& m = plans[q];
    for (int p = 0; p < 2; ++p) {
      Carve fcv = cv;  // the same fp64 workspace for every product, in stream order
      CHK(issue_fp64(c, fcv, m.M, m.N, m.K, m.K, op[q].eps, m.K, p == 0 ? op[q].g : m.t.a1, m.K,
                     p == 0 ? m.t.b0 : m.t.b1, m.N, op[q].del, m.N,
                     make_ep(p == 0 ? m.t.c0 : m.t.c1, +1, trunc, p == 0 ? m.z0 : m.z1, rowmajor_view(m.N))));
    }
  }
  return MPC_OK;
}

// Plain form: eps, g0 = a0 + eps and delta row-major; party p's finish is
// z_p = c_p + [eps | g_p] @ [b_p ; delta] with g_1 = a_1.
void matmul_plain(const MatmulPlan& m, Carve& cv, int trunc, std::vector<OpenJob>& opens,
                  std::vector<PlainProblem>& probs) {
  u64* eps = cv.take<u64>((size_t)(m.M * m.K));
  u64* g = cv.take<u64>((size_t)(m.M * m.K));
  u64* del = cv.take<u64>((size_t)(m.K * m.N));
  opens.push_back(OpenJob{kOpenLeft, m.M * m.K, m.x0, m.x1, m.t.a0, m.t.a1, eps, g});
  opens.push_back(OpenJob{kOpenRight, m.K * m.N, m.y0, m.y1, m.t.b0, m.t.b1, del, nullptr});
  for (int p = 0; p < 2; ++p)
    probs.push_back(plain_problem(m.M, m.N, m.K, m.K, eps, nullptr, m.K, p == 0 ? g : m.t.a1, m.K,
                                  p == 0 ? m.t.b0 : m.t.b1, nullptr, m.N, del, m.N,
                                  make_ep(p == 0 ? m.t.c0 : m.t.c1, +1, trunc, p == 0 ? m.z0 : m.z1,
                                          rowmajor_view(m.N))));
}

// Limb form: one fused open+pack job per operand side, then the same finish
// over packed operands.
void matmul_limb(const MatmulPlan& m, Carve& cv, int trunc, std::vector<PackJob>& jobs,
                 std::vector<LimbReq>& reqs) {
  JobSpec jl = left_job(m.M, m.K, m.K), jr = right_job(m.K, m.N, m.N);
  open_left(jl, m.x0, m.x1, m.t.a0, m.t.a1);
  open_right(jr, m.y0, m.y1, m.t.b0, m.t.b1);
  if (m.packed) {
    // a_1, b_0, b_1 come packed from the dealer: the open packs eps, g0 and
    // delta only
    jl.mode = kModeOpenLeft2;
    jr.mode = kModeOpenRight1;
    size_t off[3];
    packed_triple_layout(m.M, m.N, m.K, off);
    PackJob L = place_job(jl, cv), R = place_job(jr, cv);
    jobs.push_back(L);
    jobs.push_back(R);
    const uint8_t *a1 = m.packed + off[0], *b0 = m.packed + off[1], *b1 = m.packed + off[2];
    for (int p = 0; p < 2; ++p)
      reqs.push_back(limb_req(m.M, m.N, m.K, m.K, L.dst[0], p == 0 ? L.dst[1] : a1, p == 0 ? b0 : b1, R.dst[0],
                              make_ep(p == 0 ? m.t.c0 : m.t.c1, +1, trunc, p == 0 ? m.z0 : m.z1,
                                      rowmajor_view(m.N))));
    return;
  }
  const PackJob L = place_job(jl, cv), R = place_job(jr, cv);
  jobs.push_back(L);
  jobs.push_back(R);
  // L.dst: eps, g0, a1;  R.dst: delta, b0, b1
  for (int p = 0; p < 2; ++p)
    reqs.push_back(limb_req(m.M, m.N, m.K, m.K, L.dst[0], L.dst[p == 0 ? 1 : 2], R.dst[p == 0 ? 1 : 2],
                            R.dst[0],
                            make_ep(p == 0 ? m.t.c0 : m.t.c1, +1, trunc, p == 0 ? m.z0 : m.z1,
                                    rowmajor_view(m.N))));
}

mpc_status run_matmuls(mpc_ctx* c, const std::vector<MatmulPlan>& plans, int trunc, mpc_form form) {
  if (form == MPC_FORM_FP64LIMB) {
    CHK(run_matmuls_fp64(c, plans, trunc));
  } else if (form == MPC_FORM_LIMB8) {
    size_t need = kAlign;
    for (const MatmulPlan& m : plans) need += matmul_ws(m, form);
    CHK(ensure_ws(c, need));
    Carve cv(c->ws);
    std::vector<PackJob> jobs;
    std::vector<LimbReq> reqs;
    std::vector<std::array<i64, 3>> shapes;
    for (const MatmulPlan& m : plans) {
      matmul_limb(m, cv, trunc, jobs, reqs);
      shapes.push_back({m.M, m.N, m.K});
    }
    // every problem's two finish GEMMs take its schedule and tile class
    const std::vector<ProbSched> ts = scheds_for(c, shapes);
    for (size_t q = 0; q < reqs.size(); ++q) {
      reqs[q].own_sched = true;
      reqs[q].sched = ts[q / 2].s;
      reqs[q].cls = ts[q / 2].cls;
    }
    CHK(issue_limb(c, jobs, reqs, c->sched_default));
  } else if (plans.size() == 1 && plans[0].K <= kSmallMatmulK && plans[0].M * plans[0].N <= kSmallMatmulMacs &&
             plans[0].M * plans[0].N * plans[0].K <= kSmallMatmulMacs) {
    // a small product: open and finish in one launch, no workspace
    const MatmulPlan& m = plans[0];
    const SmallMatmul s{m.M, m.N, m.K, m.x0, m.x1, m.y0, m.y1, m.t.a0, m.t.a1, m.t.b0, m.t.b1,
                        m.t.c0, m.t.c1, m.z0, m.z1, trunc};
    CHK(hip_status(launch_beaver_matmul_small(c->s[0], s)));
    c->stats.launches++;
  } else {
    size_t need = kAlign;
    for (const MatmulPlan& m : plans) need += matmul_ws(m, form);
    CHK(ensure_ws(c, need));
    Carve cv(c->ws);
    std::vector<OpenJob> opens;
    std::vector<PlainProblem> probs;
    for (const MatmulPlan& m : plans) matmul_plain(m, cv, trunc, opens, probs);
    CHK(issue_opens(c, opens));
    CHK(issue_plain(c, probs));
  }
  for (const MatmulPlan& m : plans) {
    c->stats.opens++;
    c->stats.open_bytes_per_party += 8 * (uint64_t)(m.M * m.K + m.K * m.N);
    if (trunc) c->stats.truncations++;
  }
  return MPC_OK;
}

}  // namespace

mpc_status mpc_beaver_matmul(mpc_ctx* c, int64_t M, int64_t N, int64_t K, const uint64_t* x0,
                             const uint64_t* x1, const uint64_t* y0, const uint64_t* y1,
                             const mpc_triple* t, int trunc_bits, mpc_form form, uint64_t* z0,
                             uint64_t* z1) {
  if (!c || !t) return MPC_E_INVAL;
  CHK(check_trunc(trunc_bits));
  CHK(check_form(form));
  MatmulPlan m{M, N, K, x0, x1, y0, y1, *t, z0, z1};
  CHK(validate_matmul(m));
  form = resolve_form(form, M, N, 2 * K, K);
  CHK(check_limb_k(form, K));
  if (M == 0 || N == 0) return MPC_OK;
  CHK(set_device(c));
  CHK(run_matmuls(c, {m}, trunc_bits, form));
  return end_call(c);
}

namespace {

// Checks of an offline-packed triple buffer against a problem's outputs.
mpc_status check_packed(const void* packed, i64 M, i64 N, i64 K, const u64* z0, const u64* z1) {
  if (!packed || ((uintptr_t)packed & 255)) return MPC_E_INVAL;
  size_t off[3];
  const size_t bytes = packed_triple_layout(M, N, K, off);
  const size_t nc = (size_t)(M * N);
  // overlap() counts 8-byte elements; the packed size is whole 8 KiB blocks
  if (overlap(packed, bytes / 8, z0, nc) || overlap(packed, bytes / 8, z1, nc)) return MPC_E_ALIAS;
  return MPC_OK;
}

}  // namespace

size_t mpc_packed_triple_bytes(int64_t M, int64_t N, int64_t K) {
  if (check_mnk(M, N, K) != MPC_OK) return 0;
  size_t off[3];
  return packed_triple_layout(M, N, K, off);
}

mpc_status mpc_dealer_triples_packed(mpc_ctx* c, uint64_t dseed, uint64_t tag, int64_t M, int64_t N, int64_t K,
                                     const mpc_triple* t, void* packed) {
  if (!c || !t || !packed || ((uintptr_t)packed & 255)) return MPC_E_INVAL;
  CHK(check_mnk(M, N, K));
  CHK(check_limb_k(MPC_FORM_LIMB8, K));
  const size_t na = (size_t)(M * K), nb = (size_t)(K * N), nc = (size_t)(M * N);
  size_t off[3];
  const size_t pbytes = packed_triple_layout(M, N, K, off);
  // element counts (8 bytes each), as overlap() takes them
  const void* bufs[7] = {t->a0, t->a1, t->b0, t->b1, t->c0, t->c1, packed};
  const size_t ns[7] = {na, na, nb, nb, nc, nc, pbytes / 8};
  for (int i = 0; i < 6; ++i) CHK(check_ptr(bufs[i], ns[i]));
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < i; ++j)
      if (overlap(bufs[i], ns[i], bufs[j], ns[j])) return MPC_E_ALIAS;
  const int64_t dims[3] = {M, N, K};
  // nothing to pack: the plain triple alone
  if (!M || !N || !K) return mpc_dealer_triples(c, MPC_TRIPLE_MATMUL, dseed, tag, dims, t);
  u64 key[6];
  for (int sl = 0; sl < 6; ++sl) key[sl] = stream_key(dseed, tag, (u64)sl);
  CHK(set_device(c));
  // the same draws and the same c as mpc_dealer_triples: a_p, b_p drawn
  // inside their packs (which also pack a_1, b_0, b_1 into `packed`), c_0
  // from the PRG, c_1 = (a_0 + a_1) @ (b_0 + b_1) - c_0
  JobSpec jl = left_job(M, K, K), jr = right_job(K, N, N);
  set_prg_sum2(jl, key[kSlotA0], key[kSlotA0 + 1], t->a0, t->a1);
  set_prg_sum2(jr, key[kSlotB0], key[kSlotB0 + 1], t->b0, t->b1);
  jl.mode = kModePrgSum2A;
  jr.mode = kModePrgSum2B;
  CHK(ensure_ws(c, kAlign + align_up(packed_bytes(M, K)) + align_up(packed_bytes(N, K))));
  CHK(hip_status(launch_prg_fill(c->s[0], key[kSlotC0], t->c0, nc)));
  c->stats.launches++;
  Carve cv(c->ws);
  PackJob L = place_job(jl, cv, 1), R = place_job(jr, cv, 1);
  uint8_t* pk = (uint8_t*)packed;
  L.dst[1] = pk + off[0];
  R.dst[1] = pk + off[1];
  R.dst[2] = pk + off[2];
  const Epilogue ep = make_ep(t->c0, -1, 0, t->c1, rowmajor_view(N));
  CHK(issue_limb(c, {L, R}, {limb_req(M, N, K, 0, L.dst[0], nullptr, R.dst[0], nullptr, ep)}, c->sched_default));
  return end_call(c);
}

mpc_status mpc_beaver_matmul_prepacked(mpc_ctx* c, int64_t M, int64_t N, int64_t K, const uint64_t* x0,
                                       const uint64_t* x1, const uint64_t* y0, const uint64_t* y1,
                                       const mpc_triple* t, const void* packed, int trunc_bits, uint64_t* z0,
                                       uint64_t* z1) {
  if (!c || !t) return MPC_E_INVAL;
  CHK(check_trunc(trunc_bits));
  MatmulPlan m{M, N, K, x0, x1, y0, y1, *t, z0, z1, (const uint8_t*)packed};
  CHK(validate_matmul(m));
  CHK(check_packed(packed, M, N, K, z0, z1));
  CHK(check_limb_k(MPC_FORM_LIMB8, K));
  if (M == 0 || N == 0) return MPC_OK;
  CHK(set_device(c));
  CHK(run_matmuls(c, {m}, trunc_bits, MPC_FORM_LIMB8));
  return end_call(c);
}

mpc_status mpc_beaver_matmul_grouped_prepacked(mpc_ctx* c, size_t count, const mpc_matmul_desc* descs,
                                               const void* const* packed, int trunc_bits) {
  if (!c || (count && (!descs || !packed))) return MPC_E_INVAL;
  CHK(check_trunc(trunc_bits));
  std::vector<MatmulPlan> plans;
  i64 kmax = 0;
  std::vector<Span> outs, ins;
  for (size_t i = 0; i < count; ++i) {
    const mpc_matmul_desc& d = descs[i];
    MatmulPlan m{d.M, d.N, d.K, d.x0, d.x1, d.y0, d.y1, d.t, d.z0, d.z1, (const uint8_t*)packed[i]};
    CHK(validate_matmul(m));
    CHK(check_packed(packed[i], d.M, d.N, d.K, d.z0, d.z1));
    if (d.M == 0 || d.N == 0) continue;
    kmax = std::max(kmax, m.K);
    plans.push_back(m);
    const size_t na = (size_t)(m.M * m.K), nb = (size_t)(m.K * m.N), nc = (size_t)(m.M * m.N);
    size_t off[3];
    add_span(outs, m.z0, nc);
    add_span(outs, m.z1, nc);
    for (const void* p : {(const void*)m.x0, (const void*)m.x1, (const void*)m.t.a0, (const void*)m.t.a1})
      add_span(ins, p, na);
    for (const void* p : {(const void*)m.y0, (const void*)m.y1, (const void*)m.t.b0, (const void*)m.t.b1})
      add_span(ins, p, nb);
    add_span(ins, m.t.c0, nc);
    add_span(ins, m.t.c1, nc);
    add_span(ins, m.packed, packed_triple_layout(m.M, m.N, m.K, off) / 8);
  }
  CHK(check_limb_k(MPC_FORM_LIMB8, kmax));
  if (plans.empty()) return MPC_OK;
  CHK(batch_disjoint(std::move(outs), ins));
  CHK(set_device(c));
  std::stable_sort(plans.begin(), plans.end(), [](const MatmulPlan& a, const MatmulPlan& b) { return a.K > b.K; });
  CHK(run_matmuls(c, plans, trunc_bits, MPC_FORM_LIMB8));
  return end_call(c);
}

mpc_status mpc_beaver_matmul_noalloc(mpc_ctx* c, int64_t M, int64_t N, int64_t K, const uint64_t* x0,
                                     const uint64_t* x1, const uint64_t* y0, const uint64_t* y1,
                                     const mpc_triple* t, int trunc_bits, mpc_form form, uint64_t* z0,
                                     uint64_t* z1) {
  if (!c || !t) return MPC_E_INVAL;
  CHK(check_trunc(trunc_bits));
  CHK(check_form(form));
  if (form != MPC_FORM_LIMB8 && form != MPC_FORM_AUTO) return MPC_E_UNSUPPORTED;
  MatmulPlan m{M, N, K, x0, x1, y0, y1, *t, z0, z1};
  CHK(validate_matmul(m));
  CHK(check_limb_k(MPC_FORM_LIMB8, K));
  if (matmul_ws(m, MPC_FORM_LIMB8) > kNoAllocBytes) return MPC_E_SHAPE;
  if (M == 0 || N == 0) return MPC_OK;
  if (!c->scratch) return MPC_E_HIP;
  CHK(set_device(c));
  if (form == MPC_FORM_AUTO && resolve_form(form, M, N, 2 * K, K) == MPC_FORM_PLAIN && K <= kSmallMatmulK &&
      M * N <= kSmallMatmulMacs && M * N * K <= kSmallMatmulMacs) {
    // a small product: open and finish in one launch, no workspace at all
    const SmallMatmul s{M, N, K, x0, x1, y0, y1, t->a0, t->a1, t->b0, t->b1, t->c0, t->c1, z0, z1, trunc_bits};
    CHK(hip_status(launch_beaver_matmul_small(c->s[0], s)));
    c->stats.launches++;
  } else {
    // the limb form over `scratch`: descriptor tables inline, no split-K
    Carve cv(c->scratch);
    std::vector<PackJob> jobs;
    std::vector<LimbReq> reqs;
    matmul_limb(m, cv, trunc_bits, jobs, reqs);
    const ProbSched ts = scheds_for(c, {{M, N, K}})[0];
    for (LimbReq& r : reqs) r.cls = ts.cls;
    CHK(issue_limb(c, jobs, reqs, ts.s, true));
  }
  c->stats.opens++;
  c->stats.open_bytes_per_party += 8 * (uint64_t)(M * K + K * N);
  if (trunc_bits) c->stats.truncations++;
  return end_call(c);
}

mpc_status mpc_beaver_conv1d(mpc_ctx* c, const mpc_conv1d_shape* shape, const uint64_t* x0,
                             const uint64_t* x1, const uint64_t* w0, const uint64_t* w1,
                             const mpc_triple* t, int trunc_bits, mpc_form form, uint64_t* z0,
                             uint64_t* z1) {
  if (!c || !t) return MPC_E_INVAL;
  CHK(check_conv(shape));
  CHK(check_trunc(trunc_bits));
  CHK(check_form(form));
  const mpc_conv1d_shape s = *shape;
  const i64 lout = conv_lout(s);
  const size_t nx = (size_t)(s.batch * s.cin * s.length), nw = (size_t)(s.cout * s.cin * s.ksize);
  const size_t ny = (size_t)(s.batch * s.cout * lout);
  const void* in[10] = {x0, x1, w0, w1, t->a0, t->a1, t->b0, t->b1, t->c0, t->c1};
  const size_t ns[10] = {nx, nx, nw, nw, nx, nx, nw, nw, ny, ny};
  for (int i = 0; i < 10; ++i) CHK(check_ptr(in[i], ns[i]));
  CHK(check_ptr(z0, ny));
  CHK(check_ptr(z1, ny));
  if (overlap(z0, ny, z1, ny)) return MPC_E_ALIAS;
  for (int i = 0; i < 10; ++i)
    if (overlap(z0, ny, in[i], ns[i]) || overlap(z1, ny, in[i], ns[i])) return MPC_E_ALIAS;
  if (ny == 0) return MPC_OK;
  CHK(set_device(c));
  // transposed orientation: z_p[b][o][l] is element (o, b*Lout + l) of
  //   c_p + Wm(b_p) @ im2col(eps) + Wm(delta) @ im2col(g_p),  g_0 = a_0 + eps, g_1 = a_1
  const i64 M = s.cout, N = s.batch * lout, K = s.cin * s.ksize;
  form = resolve_form(form, M, N, 2 * K, K);
  CHK(check_limb_k(form, K));
  const OutView view{lout, std::max<i64>(lout, 1), s.cout * lout};
  if (form == MPC_FORM_LIMB8) {
    JobSpec jw = left_job(M, K, K), jx = im2col_job(s, lout);
    open_right(jw, w0, w1, t->b0, t->b1);  // delta, b0, b1 (weights)
    open_left(jx, x0, x1, t->a0, t->a1);   // im2col of eps, g0, a1 (activations)
    CHK(ensure_ws(c, kAlign + job_bytes(jw) + job_bytes(jx)));
    Carve cv(c->ws);
    const PackJob W = place_job(jw, cv), X = place_job(jx, cv);
    std::vector<LimbReq> reqs;
    for (int p = 0; p < 2; ++p)
      reqs.push_back(limb_req(M, N, K, K, W.dst[p == 0 ? 1 : 2], W.dst[0], X.dst[0], X.dst[p == 0 ? 1 : 2],
                              make_ep(p == 0 ? t->c0 : t->c1, +1, trunc_bits, p == 0 ? z0 : z1, view)));
    CHK(issue_limb(c, {W, X}, reqs, c->sched_default));
  } else {
    // plain and fp64 limb forms: open, then im2col of eps, g_0 and a_1 into
    // row-major K x N matrices
    const size_t kn = (size_t)(K * N);
    const bool fp = form == MPC_FORM_FP64LIMB;
    if (fp && 2 * K >= kFp64MaxK) return MPC_E_UNSUPPORTED;
    if (fp) CHK(fp64_ready(c));
    CHK(ensure_ws(c, kAlign + 2 * align_up(nx * 8) + align_up(nw * 8) + 3 * align_up(kn * 8) +
                         (fp ? fp64_ws(M, N, 2 * K) : 0)));
    Carve cv(c->ws);
    u64* eps = cv.take<u64>(nx);
    u64* g = cv.take<u64>(nx);
    u64* del = cv.take<u64>(nw);
    u64* col_e = cv.take<u64>(kn);
    u64* col_g = cv.take<u64>(kn);
    u64* col_a1 = cv.take<u64>(kn);
    CHK(issue_opens(c, {OpenJob{kOpenLeft, (i64)nx, x0, x1, t->a0, t->a1, eps, g},
                        OpenJob{kOpenRight, (i64)nw, w0, w1, t->b0, t->b1, del, nullptr}}));
    hipStream_t st = c->s[0];
    CHK(hip_status(launch_im2col(st, eps, nullptr, s.batch, s.cin, s.length, s.ksize, s.stride, lout, col_e)));
    CHK(hip_status(launch_im2col(st, g, nullptr, s.batch, s.cin, s.length, s.ksize, s.stride, lout, col_g)));
    CHK(hip_status(launch_im2col(st, t->a1, nullptr, s.batch, s.cin, s.length, s.ksize, s.stride, lout, col_a1)));
    c->stats.launches += 3;
    if (fp) {
      // each party's [Wm(b_p) | Wm(delta)] @ [im2col(eps) ; im2col(g_p)], one
      // after the other through one fp64 workspace
      for (int p = 0; p < 2; ++p) {
        Carve fcv = cv;
        CHK(issue_fp64(c, fcv, M, N, K, K, p == 0 ? t->b0 : t->b1, K, del, K, col_e, N, p == 0 ? col_g : col_a1,
                       N, make_ep(p == 0 ? t->c0 : t->c1, +1, trunc_bits, p == 0 ? z0 : z1, view)));
      }
    } else {
      std::vector<PlainProblem> probs;
      for (int p = 0; p < 2; ++p)
        probs.push_back(plain_problem(M, N, K, K, p == 0 ? t->b0 : t->b1, nullptr, K, del, K, col_e, nullptr, N,
                                      p == 0 ? col_g : col_a1, N,
                                      make_ep(p == 0 ? t->c0 : t->c1, +1, trunc_bits, p == 0 ? z0 : z1, view)));
      CHK(issue_plain(c, probs));
    }
  }
  c->stats.opens++;
  c->stats.open_bytes_per_party += 8 * (uint64_t)(nx + nw);
  if (trunc_bits) c->stats.truncations++;
  return end_call(c);
}

mpc_status mpc_ring_gemm(mpc_ctx* c, int64_t M, int64_t N, int64_t K, const uint64_t* A,
                         const uint64_t* B, uint64_t* C, mpc_form form) {
  if (!c) return MPC_E_INVAL;
  CHK(check_form(form));
  CHK(check_mnk(M, N, K));
  CHK(check_ptr(A, (size_t)(M * K)));
  CHK(check_ptr(B, (size_t)(K * N)));
  CHK(check_ptr(C, (size_t)(M * N)));
  if (overlap(C, (size_t)(M * N), A, (size_t)(M * K)) || overlap(C, (size_t)(M * N), B, (size_t)(K * N)))
    return MPC_E_ALIAS;
  if (M == 0 || N == 0) return MPC_OK;
  CHK(set_device(c));
  form = resolve_form(form, M, N, K, K);
  CHK(check_limb_k(form, K));
  const Epilogue ep = make_ep(nullptr, +1, 0, C, rowmajor_view(N));
  if (form == MPC_FORM_LIMB8) {
    JobSpec ja = left_job(M, K, K), jb = right_job(K, N, N);
    set_mode(ja, kModeCopy, {A});
    set_mode(jb, kModeCopy, {B});
    CHK(ensure_ws(c, kAlign + job_bytes(ja) + job_bytes(jb)));
    Carve cv(c->ws);
    const PackJob PA = place_job(ja, cv), PB = place_job(jb, cv);
    CHK(issue_limb(c, {PA, PB}, {limb_req(M, N, K, 0, PA.dst[0], nullptr, PB.dst[0], nullptr, ep)}, c->sched_default));
  } else if (form == MPC_FORM_FP64LIMB) {
    if (K >= kFp64MaxK) return MPC_E_UNSUPPORTED;
    CHK(ensure_ws(c, kAlign + fp64_ws(M, N, K)));
    Carve cv(c->ws);
    CHK(issue_fp64(c, cv, M, N, K, 0, A, K, nullptr, 0, B, N, nullptr, 0, ep));
  } else {
    CHK(issue_plain(c, {plain_problem(M, N, K, 0, A, nullptr, K, nullptr, 0, B, nullptr, N, nullptr, 0, ep)}));
  }
  return end_call(c);
}

mpc_status mpc_beaver_matmul_grouped(mpc_ctx* c, size_t count, const mpc_matmul_desc* descs,
                                     int trunc_bits, mpc_form form) {
  if (!c || (count && !descs)) return MPC_E_INVAL;
  CHK(check_trunc(trunc_bits));
  CHK(check_form(form));
  std::vector<MatmulPlan> plans;
  for (size_t i = 0; i < count; ++i) {
    const mpc_matmul_desc& d = descs[i];
    MatmulPlan m{d.M, d.N, d.K, d.x0, d.x1, d.y0, d.y1, d.t, d.z0, d.z1};
    CHK(validate_matmul(m));
    if (d.M == 0 || d.N == 0) continue;
    plans.push_back(m);
  }
  // AUTO: the limb form, unless a problem's k is longer than it addresses
  i64 kmax = 0;
  for (const MatmulPlan& m : plans) kmax = std::max(kmax, m.K);
  if (form == MPC_FORM_AUTO) form = kmax > kLimbMaxSegK ? MPC_FORM_PLAIN : MPC_FORM_LIMB8;
  CHK(check_limb_k(form, kmax));
  if (plans.empty()) return MPC_OK;
  {
    std::vector<Span> outs, ins;
    for (const MatmulPlan& m : plans) {
      const size_t na = (size_t)(m.M * m.K), nb = (size_t)(m.K * m.N), nc = (size_t)(m.M * m.N);
      add_span(outs, m.z0, nc);
      add_span(outs, m.z1, nc);
      for (const void* p : {(const void*)m.x0, (const void*)m.x1, (const void*)m.t.a0, (const void*)m.t.a1})
        add_span(ins, p, na);
      for (const void* p : {(const void*)m.y0, (const void*)m.y1, (const void*)m.t.b0, (const void*)m.t.b1})
        add_span(ins, p, nb);
      add_span(ins, m.t.c0, nc);
      add_span(ins, m.t.c1, nc);
    }
    CHK(batch_disjoint(std::move(outs), ins));
  }
  CHK(set_device(c));
  // heavy problems first, so the GEMM's tile list front-loads the long tiles
  std::stable_sort(plans.begin(), plans.end(), [](const MatmulPlan& a, const MatmulPlan& b) {
    return a.K > b.K;
  });
  CHK(run_matmuls(c, plans, trunc_bits, form));
  return end_call(c);
}

mpc_status mpc_beaver_mul_grouped(mpc_ctx* c, size_t count, const mpc_mul_desc* descs, int trunc_bits) {
  if (!c || (count && !descs)) return MPC_E_INVAL;
  CHK(check_trunc(trunc_bits));
  std::vector<MulJob> jobs;
  uint64_t open_bytes = 0;
  for (size_t i = 0; i < count; ++i) {
    const mpc_mul_desc& d = descs[i];
    const bool sq = d.y0 == nullptr && d.y1 == nullptr;
    if (!sq && (d.y0 == nullptr || d.y1 == nullptr)) return MPC_E_INVAL;
    const size_t n = d.n;
    const void* in[10] = {d.x0, d.x1, d.y0, d.y1, d.t.a0, d.t.a1, d.t.b0, d.t.b1, d.t.c0, d.t.c1};
    const int nin = sq ? 8 : 10;
    for (int k = 0; k < nin; ++k) {
      if (sq && (k == 2 || k == 3)) continue;
      CHK(check_ptr(in[k], n));
    }
    CHK(check_ptr(d.z0, n));
    CHK(check_ptr(d.z1, n));
    if (overlap(d.z0, n, d.z1, n)) return MPC_E_ALIAS;
    for (int k = 0; k < nin; ++k)
      if (overlap(d.z0, n, in[k], n) || overlap(d.z1, n, in[k], n)) return MPC_E_ALIAS;
    if (!n) continue;
    MulJob j{};
    j.n = (i64)n;
    j.x0 = d.x0;
    j.x1 = d.x1;
    j.y0 = sq ? nullptr : d.y0;
    j.y1 = sq ? nullptr : d.y1;
    j.a0 = d.t.a0;
    j.a1 = d.t.a1;
    j.b0 = d.t.b0;
    j.b1 = d.t.b1;
    j.c0 = sq ? nullptr : d.t.c0;
    j.c1 = sq ? nullptr : d.t.c1;
    j.z0 = d.z0;
    j.z1 = d.z1;
    bool al = true;
    for (const void* p : {(const void*)j.x0, (const void*)j.x1, (const void*)j.y0, (const void*)j.y1,
                          (const void*)j.a0, (const void*)j.a1, (const void*)j.b0, (const void*)j.b1,
                          (const void*)j.c0, (const void*)j.c1, (const void*)j.z0, (const void*)j.z1})
      if (((uintptr_t)p & 15) != 0) al = false;
    j.vec2 = al ? 1 : 0;
    jobs.push_back(j);
    open_bytes += (sq ? 1 : 2) * 8 * (uint64_t)n;
  }
  if (jobs.empty()) return MPC_OK;
  {
    std::vector<Span> outs, ins;
    for (const MulJob& j : jobs) {
      add_span(outs, j.z0, (size_t)j.n);
      add_span(outs, j.z1, (size_t)j.n);
      for (const void* p : {(const void*)j.x0, (const void*)j.x1, (const void*)j.y0, (const void*)j.y1,
                            (const void*)j.a0, (const void*)j.a1, (const void*)j.b0, (const void*)j.b1,
                            (const void*)j.c0, (const void*)j.c1})
        add_span(ins, p, (size_t)j.n);
    }
    CHK(batch_disjoint(std::move(outs), ins));
  }
  CHK(set_device(c));
  std::vector<i64> cs(jobs.size() + 1, 0);
  for (size_t i = 0; i < jobs.size(); ++i) cs[i + 1] = cs[i] + (jobs[i].n + kMulChunk - 1) / kMulChunk;
  Blob blob;
  const size_t ojobs = blob.add(jobs.data(), jobs.size());
  const size_t ostart = blob.add(cs.data(), cs.size());
  uint8_t* dev = nullptr;
  CHK(upload(c, blob, &dev));
  CHK(hip_status(launch_beaver_mul_grouped(c->s[0], (const MulJob*)(dev + ojobs), (const i64*)(dev + ostart),
                                           (int)jobs.size(), cs.back(), trunc_bits)));
  c->stats.launches++;
  c->stats.opens += jobs.size();  // one open per product, all in the same round
  c->stats.open_bytes_per_party += open_bytes;
  if (trunc_bits) c->stats.truncations += jobs.size();
  return end_call(c);
}

// ------------------------------------------------------------------ autotuning
mpc_status mpc_autotune_matmul(mpc_ctx* c, size_t count, const int64_t* dims, mpc_tile_config* best) {
  if (!c || (count && !dims) || c->capturing) return MPC_E_INVAL;
  std::vector<std::array<i64, 3>> shapes;
  for (size_t i = 0; i < count; ++i) {
    const i64 M = dims[3 * i], N = dims[3 * i + 1], K = dims[3 * i + 2];
    CHK(check_mnk(M, N, K));
    CHK(check_limb_k(MPC_FORM_LIMB8, K));
    if (M && N) shapes.push_back({M, N, K});
  }
  if (shapes.empty()) return MPC_OK;
  CHK(set_device(c));
  // the order a grouped call issues its problems in
  if (shapes.size() > 1)
    std::stable_sort(shapes.begin(), shapes.end(),
                     [](const std::array<i64, 3>& a, const std::array<i64, 3>& b) { return a[2] > b[2]; });
  // packed operands of both parties' finish GEMMs, as a Beaver matmul lays
  // them out: left eps, g0, a1 and right delta, b0, b1 per problem
  size_t need = kAlign;
  for (const auto& s : shapes)
    need += 3 * align_up(packed_bytes(s[0], s[2])) + 3 * align_up(packed_bytes(s[1], s[2]));
  CHK(ensure_ws(c, need));
  Carve cv(c->ws);
  std::vector<LimbReq> reqs[kBuckets];
  for (const auto& s : shapes) {
    const i64 M = s[0], N = s[1], K = s[2];
    uint8_t* L[3];
    uint8_t* R[3];
    for (auto& p : L) p = cv.take<uint8_t>(packed_bytes(M, K));
    for (auto& p : R) p = cv.take<uint8_t>(packed_bytes(N, K));
    for (int p = 0; p < 2; ++p)
      reqs[bucket_of(M, N)].push_back(limb_req(M, N, K, K, L[0], L[p == 0 ? 1 : 2], R[p == 0 ? 1 : 2], R[0],
                                               make_ep(nullptr, +1, 0, nullptr, rowmajor_view(N))));
  }
  for (int b = 0; b < kBuckets; ++b)
    for (LimbReq& r : reqs[b]) r.cls = b;
  // random limbs: the matrix cores' power draw, and so their clock, depends
  // on the data
  CHK(hip_status(launch_prg_fill(c->s[0], stream_key(c->seed, 0x7475, 0), (u64*)c->ws, cv.off / 8)));
  // outputs: one scratch buffer per party, the largest problem's size
  i64 maxmn = 0;
  for (const auto& s : shapes) maxmn = std::max(maxmn, s[0] * s[1]);
  u64* out[2] = {nullptr, nullptr};
  for (int p = 0; p < 2; ++p) HIPCHK(hipMalloc((void**)&out[p], (size_t)maxmn * 8));
  for (auto& rb : reqs)
    for (size_t q = 0; q < rb.size(); ++q) rb[q].ep.Out = out[q & 1];
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const bool prof = c->profiling;
  c->profiling = false;
  mpc_status st = MPC_OK;
  // mean time of `reps` issues of a request list under one schedule
  auto time_reqs = [&](const std::vector<LimbReq>& rq, const TileSched& ts, double* ms_out) -> mpc_status {
    CHK(issue_limb(c, {}, rq, ts));  // warm-up
    CHK(mark_slot(c));
    const int reps = 3;
    HIPCHK(hipEventRecord(e0, c->s[0]));
    for (int r = 0; r < reps; ++r) {
      CHK(issue_limb(c, {}, rq, ts));
      CHK(mark_slot(c));
    }
    HIPCHK(hipEventRecord(e1, c->s[0]));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    *ms_out = ms / reps;
    return MPC_OK;
  };
  // every class on its own: all schedules on that class's GEMMs alone (one
  // launch per class when the classes end up with different schedules)
  const TileSched d = c->sched_default;
  BucketScheds tuned{{d, d, d}};
  mpc_tile_config win[kBuckets];
  double split_ms = 0;
  for (int b = 0; b < kBuckets && st == MPC_OK; ++b) {
    win[b] = mpc_tile_config{d.variant, d.group_m, d.xcd_remap, 0.0};
    if (reqs[b].empty()) continue;
    win[b].ms = 1e30;
    for (int v = 0; v < kLimbVariants && st == MPC_OK; ++v)
      for (int gm : {4, 8, 16})
        for (int remap : {1, 0}) {
          double ms = 0;
          st = time_reqs(reqs[b], TileSched{v, gm, remap}, &ms);
          if (st != MPC_OK) break;
          if (ms < win[b].ms) win[b] = mpc_tile_config{v, gm, remap, ms};
        }
    tuned.s[b] = TileSched{win[b].variant, win[b].group_m, win[b].xcd_remap};
    split_ms += win[b].ms;
  }
  // and every problem in one launch: under each single schedule, and under
  // the classes schedule with its own tile class
  std::vector<LimbReq> all;
  for (const auto& rb : reqs) all.insert(all.end(), rb.begin(), rb.end());
  int nclasses = 0;
  for (const auto& rb : reqs) nclasses += rb.empty() ? 0 : 1;
  if (st == MPC_OK && nclasses > 1)
    for (int v = 0; v < kLimbVariants && st == MPC_OK; ++v)
      for (int gm : {4, 8, 16})
        for (int remap : {1, 0}) {
          double ms = 0;
          st = time_reqs(all, TileSched{v, gm, remap}, &ms);
          if (st != MPC_OK) break;
          if (ms < split_ms) {
            split_ms = ms;
            for (int b = 0; b < kBuckets; ++b) {
              tuned.s[b] = TileSched{v, gm, remap};
              if (!reqs[b].empty()) win[b] = mpc_tile_config{v, gm, remap, 0.0};
            }
            // the launch's time, charged to the regular class
            win[kBucketRegular].ms = ms;
          }
        }
  c->profiling = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(c->s[0]);
  for (int p = 0; p < 2; ++p) (void)hipFree(out[p]);
  CHK(st);
  c->tuned[shapes_key(shapes)] = tuned;
  if (best) {
    // the class that takes longest, with the time of all classes
    int top = 0;
    double total = 0;
    for (int b = 0; b < kBuckets; ++b) {
      total += win[b].ms;
      if (win[b].ms > win[top].ms) top = b;
    }
    *best = win[top];
    best->ms = total;
  }
  return end_call(c);
}

mpc_status mpc_autotune_save(const mpc_ctx* c, const char* path) {
  if (!c || !path) return MPC_E_INVAL;
  FILE* f = std::fopen(path, "w");
  if (!f) return MPC_E_INVAL;
  for (const auto& kv : c->tuned) {
    std::fprintf(f, "%016llx", (unsigned long long)kv.first);
    for (const TileSched& t : kv.second.s) std::fprintf(f, " %d %d %d", t.variant, t.group_m, t.xcd_remap);
    std::fprintf(f, "\n");
  }
  std::fclose(f);
  return MPC_OK;
}

mpc_status mpc_autotune_load(mpc_ctx* c, const char* path) {
  if (!c || !path) return MPC_E_INVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return MPC_E_INVAL;
  unsigned long long key;
  int v[kBuckets], gm[kBuckets], remap[kBuckets];
  while (std::fscanf(f, "%llx %d %d %d %d %d %d %d %d %d", &key, &v[0], &gm[0], &remap[0], &v[1], &gm[1], &remap[1],
                     &v[2], &gm[2], &remap[2]) == 10) {
    bool ok = true;
    BucketScheds b;
    for (int i = 0; i < kBuckets; ++i) {
      ok = ok && sched_ok(v[i], gm[i]);
      b.s[i] = TileSched{v[i], gm[i], remap[i] ? 1 : 0};
    }
    if (ok) c->tuned[(uint64_t)key] = b;
  }
  std::fclose(f);
  return MPC_OK;
}

mpc_status mpc_get_default_tile_config(const mpc_ctx* c, mpc_tile_config* cfg) {
  if (!c || !cfg) return MPC_E_INVAL;
  *cfg = mpc_tile_config{c->sched_default.variant, c->sched_default.group_m, c->sched_default.xcd_remap, 0.0};
  return MPC_OK;
}

mpc_status mpc_set_default_tile_config(mpc_ctx* c, const mpc_tile_config* cfg) {
  if (!c || !cfg || !sched_ok(cfg->variant, cfg->group_m)) return MPC_E_INVAL;
  c->sched_default = TileSched{cfg->variant, cfg->group_m, cfg->xcd_remap ? 1 : 0};
  // an explicit schedule applies to thin products too
  c->class_tiles = false;
  return MPC_OK;
}

mpc_status mpc_limb_plan(int64_t M, int64_t N, int variant, int* cls, int64_t* regions, int* count,
                         int64_t* tiles) {
  if (!cls || !regions || !count || variant < 0 || variant >= kLimbVariants) return MPC_E_INVAL;
  if (M < 1 || N < 1 || !count_ok(M, N)) return MPC_E_SHAPE;
  *cls = bucket_of(M, N);
  const bool per_class = limb_per_class(variant);
  const std::vector<Region> g = limb_regions(M, N, per_class ? *cls : 0, variant, true);
  i64 nt = 0;
  for (size_t i = 0; i < g.size(); ++i) {
    int bm = limb_variant_bm(variant), bn = limb_variant_bn(variant);
    if (per_class) limb_class_shape(g[i].cls, &bm, &bn);
    const int64_t row[6] = {g[i].r0, g[i].c0, g[i].m, g[i].n, bm, bn};
    for (int k = 0; k < 6; ++k) regions[6 * i + k] = row[k];
    nt += ((g[i].m + bm - 1) / bm) * ((g[i].n + bn - 1) / bn);
  }
  *count = (int)g.size();
  if (tiles) *tiles = nt;
  return MPC_OK;
}

// ------------------------------------------------------------------ measurement
mpc_status mpc_profile_enable(mpc_ctx* c, int on) {
  if (!c) return MPC_E_INVAL;
  c->profiling = on != 0;
  return MPC_OK;
}

mpc_status mpc_profile_read(mpc_ctx* c, mpc_gemm_timing* limb8, mpc_gemm_timing* plain,
                            mpc_gemm_timing* fp64limb) {
  if (!c) return MPC_E_INVAL;
  CHK(set_device(c));
  CHK(sync_all(c));
  // [0] plain, [1] limb8, [2] fp64 limb
  mpc_gemm_timing acc[3] = {{0, 0.0, 0.0}, {0, 0.0, 0.0}, {0, 0.0, 0.0}};
  for (auto& t : c->timed) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t.start, t.stop));
    mpc_gemm_timing& a = acc[t.form == MPC_FORM_LIMB8 ? 1 : t.form == MPC_FORM_FP64LIMB ? 2 : 0];
    a.launches++;
    a.total_ms += ms;
    a.ring_macs += t.ring_macs;
    c->event_pool.push_back(t.start);
    c->event_pool.push_back(t.stop);
  }
  c->timed.clear();
  if (limb8) *limb8 = acc[1];
  if (plain) *plain = acc[0];
  if (fp64limb) *fp64limb = acc[2];
  return MPC_OK;
}

// ------------------------------------------------------------------ binary sharing
}  // extern "C"

namespace {

// The six arrays of a triple, each checked for n words.
mpc_status triple_ptrs(const mpc_triple* t, size_t n, TriplePtrs* out) {
  if (!t) return MPC_E_INVAL;
  const u64* v[6] = {t->a0, t->a1, t->b0, t->b1, t->c0, t->c1};
  for (int i = 0; i < 6; ++i) CHK(check_ptr(v[i], n));
  *out = TriplePtrs{v[0], v[1], v[2], v[3], v[4], v[5]};
  return MPC_OK;
}

// output pair against a list of (pointer, length) inputs
mpc_status out_alias(const u64* z0, const u64* z1, size_t nz, std::initializer_list<std::pair<const void*, size_t>> ins) {
  if (overlap(z0, nz, z1, nz)) return MPC_E_ALIAS;
  for (const auto& in : ins)
    if (in.first && (overlap(z0, nz, in.first, in.second) || overlap(z1, nz, in.first, in.second)))
      return MPC_E_ALIAS;
  return MPC_OK;
}

}  // namespace

extern "C" {

mpc_status mpc_bin_share(mpc_ctx* c, const uint64_t* x, size_t n, int src, uint64_t tag, uint64_t* s0,
                         uint64_t* s1) {
  if (!c || (src != 0 && src != 1)) return MPC_E_INVAL;
  CHK(check_ptr(x, n));
  CHK(check_ptr(s0, n));
  CHK(check_ptr(s1, n));
  CHK(out_alias(s0, s1, n, {{x, n}}));
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_bin_share(c->s[0], x, n, src, stream_key(c->seed, tag, kBinShare), s0, s1)));
  c->stats.launches++;
  return MPC_OK;
}

mpc_status mpc_bin_reveal(mpc_ctx* c, const uint64_t* s0, const uint64_t* s1, size_t n, uint64_t* out) {
  if (!c) return MPC_E_INVAL;
  CHK(check_ptr(s0, n));
  CHK(check_ptr(s1, n));
  CHK(check_ptr(out, n));
  if (overlap(out, n, s0, n) || overlap(out, n, s1, n)) return MPC_E_ALIAS;
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_bin_reveal(c->s[0], s0, s1, n, out)));
  c->stats.launches++;
  c->stats.opens++;
  c->stats.open_bytes_per_party += 8 * (uint64_t)n;
  return MPC_OK;
}

mpc_status mpc_dealer_and_triples(mpc_ctx* c, uint64_t dseed, uint64_t tag, size_t n, const mpc_triple* t) {
  if (!c || !t) return MPC_E_INVAL;
  TriplePtrs tp;
  CHK(triple_ptrs(t, n, &tp));
  const u64* v[6] = {tp.a0, tp.a1, tp.b0, tp.b1, tp.c0, tp.c1};
  for (int i = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j)
      if (overlap(v[i], n, v[j], n)) return MPC_E_ALIAS;
  if (!n) return MPC_OK;
  CHK(set_device(c));
  const BinKeys k{stream_key(dseed, tag, kBinA0), stream_key(dseed, tag, kBinA1), stream_key(dseed, tag, kBinB0),
                  stream_key(dseed, tag, kBinB1), stream_key(dseed, tag, kBinC0)};
  CHK(hip_status(launch_dealer_and(c->s[0], k, n, t->a0, t->a1, t->b0, t->b1, t->c0, t->c1)));
  c->stats.launches++;
  return MPC_OK;
}

mpc_status mpc_bin_and(mpc_ctx* c, size_t n, const uint64_t* x0, const uint64_t* x1, const uint64_t* y0,
                       const uint64_t* y1, const mpc_triple* t, uint64_t* z0, uint64_t* z1) {
  if (!c) return MPC_E_INVAL;
  TriplePtrs tp;
  CHK(triple_ptrs(t, n, &tp));
  const u64* in[4] = {x0, x1, y0, y1};
  for (const u64* p : in) CHK(check_ptr(p, n));
  CHK(check_ptr(z0, n));
  CHK(check_ptr(z1, n));
  CHK(out_alias(z0, z1, n, {{x0, n}, {x1, n}, {y0, n}, {y1, n}, {tp.a0, n}, {tp.a1, n}, {tp.b0, n}, {tp.b1, n},
                            {tp.c0, n}, {tp.c1, n}}));
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_bin_and(c->s[0], n, x0, x1, y0, y1, tp, z0, z1)));
  c->stats.launches++;
  c->stats.opens++;
  c->stats.open_bytes_per_party += 16 * (uint64_t)n;
  return MPC_OK;
}

mpc_status mpc_a2b(mpc_ctx* c, size_t n, const uint64_t* x0, const uint64_t* x1, uint64_t tag,
                   const mpc_triple* t, uint64_t* z0, uint64_t* z1) {
  if (!c) return MPC_E_INVAL;
  const size_t nt = (size_t)kA2bTriples * n;
  TriplePtrs tp;
  CHK(triple_ptrs(t, nt, &tp));
  CHK(check_ptr(x0, n));
  CHK(check_ptr(x1, n));
  CHK(check_ptr(z0, n));
  CHK(check_ptr(z1, n));
  CHK(out_alias(z0, z1, n, {{x0, n}, {x1, n}, {tp.a0, nt}, {tp.a1, nt}, {tp.b0, nt}, {tp.b1, nt}, {tp.c0, nt},
                            {tp.c1, nt}}));
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_a2b(c->s[0], n, x0, x1, stream_key(c->seed, tag, kA2bY0), stream_key(c->seed, tag, kA2bY1),
                            tp, z0, z1)));
  c->stats.launches++;
  c->stats.opens += 7;
  c->stats.open_bytes_per_party += 16 * (uint64_t)nt;
  return MPC_OK;
}

mpc_status mpc_dealer_b2a(mpc_ctx* c, uint64_t dseed, uint64_t tag, size_t n, uint64_t* rb0, uint64_t* rb1,
                          uint64_t* ra0, uint64_t* ra1) {
  if (!c) return MPC_E_INVAL;
  u64* v[4] = {rb0, rb1, ra0, ra1};
  for (int i = 0; i < 4; ++i) CHK(check_ptr(v[i], n));
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (overlap(v[i], n, v[j], n)) return MPC_E_ALIAS;
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_dealer_b2a(c->s[0], n, stream_key(dseed, tag, kB2aR), stream_key(dseed, tag, kB2aRb0),
                                   stream_key(dseed, tag, kB2aRa0), rb0, rb1, ra0, ra1)));
  c->stats.launches++;
  return MPC_OK;
}

mpc_status mpc_b2a_bit(mpc_ctx* c, size_t n, int bit, const uint64_t* b0, const uint64_t* b1,
                       const uint64_t* rb0, const uint64_t* rb1, const uint64_t* ra0, const uint64_t* ra1,
                       uint64_t* z0, uint64_t* z1) {
  if (!c || bit < 0 || bit > 63) return MPC_E_INVAL;
  const u64* in[6] = {b0, b1, rb0, rb1, ra0, ra1};
  for (const u64* p : in) CHK(check_ptr(p, n));
  CHK(check_ptr(z0, n));
  CHK(check_ptr(z1, n));
  CHK(out_alias(z0, z1, n, {{b0, n}, {b1, n}, {rb0, n}, {rb1, n}, {ra0, n}, {ra1, n}}));
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_b2a_bit(c->s[0], n, bit, b0, b1, rb0, rb1, ra0, ra1, z0, z1)));
  c->stats.launches++;
  c->stats.opens++;
  c->stats.open_bytes_per_party += 8 * (uint64_t)n;
  return MPC_OK;
}

mpc_status mpc_relu(mpc_ctx* c, size_t n, const uint64_t* x0, const uint64_t* x1, uint64_t tag,
                    const mpc_triple* t, const uint64_t* rb0, const uint64_t* rb1, const uint64_t* ra0,
                    const uint64_t* ra1, const mpc_triple* m, uint64_t* z0, uint64_t* z1) {
  if (!c) return MPC_E_INVAL;
  const size_t nt = (size_t)kA2bTriples * n;
  TriplePtrs tp, mp;
  CHK(triple_ptrs(t, nt, &tp));
  CHK(triple_ptrs(m, n, &mp));
  const u64* in[6] = {x0, x1, rb0, rb1, ra0, ra1};
  for (const u64* p : in) CHK(check_ptr(p, n));
  CHK(check_ptr(z0, n));
  CHK(check_ptr(z1, n));
  CHK(out_alias(z0, z1, n, {{x0, n}, {x1, n}, {rb0, n}, {rb1, n}, {ra0, n}, {ra1, n}, {tp.a0, nt}, {tp.a1, nt},
                            {tp.b0, nt}, {tp.b1, nt}, {tp.c0, nt}, {tp.c1, nt}, {mp.a0, n}, {mp.a1, n},
                            {mp.b0, n}, {mp.b1, n}, {mp.c0, n}, {mp.c1, n}}));
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_relu(c->s[0], n, x0, x1, stream_key(c->seed, tag, kA2bY0), stream_key(c->seed, tag, kA2bY1),
                             tp, rb0, rb1, ra0, ra1, mp, z0, z1)));
  c->stats.launches++;
  c->stats.opens += 9;
  c->stats.open_bytes_per_party += 16 * (uint64_t)nt + 8 * (uint64_t)n + 16 * (uint64_t)n;
  return MPC_OK;
}

// ------------------------------------------------------------------ more than two parties
}  // extern "C"

namespace {

mpc_status check_parties(int P) { return (P < 2 || P > kMaxParties) ? MPC_E_INVAL : MPC_OK; }

MpKeys mp_keys(u64 seed, u64 tag, u64 base, int P) {
  MpKeys k{};
  for (int p = 0; p < P; ++p) k.k[p] = stream_key(seed, tag, base + (u64)p);
  return k;
}

// Gathers a host array of P device pointers, each checked for n elements.
mpc_status mp_out(uint64_t* const* v, int P, size_t n, MpOut* o) {
  if (!v) return MPC_E_INVAL;
  *o = MpOut{};
  for (int p = 0; p < P; ++p) {
    CHK(check_ptr(v[p], n));
    o->p[p] = v[p];
  }
  return MPC_OK;
}
mpc_status mp_in(const uint64_t* const* v, int P, size_t n, MpIn* o) {
  if (!v) return MPC_E_INVAL;
  *o = MpIn{};
  for (int p = 0; p < P; ++p) {
    CHK(check_ptr(v[p], n));
    o->p[p] = v[p];
  }
  return MPC_OK;
}

// outputs (P buffers of no) against each other and against every input set
mpc_status mp_alias(const MpOut& out, int P, size_t no, std::initializer_list<std::pair<const MpIn*, size_t>> ins) {
  for (int p = 0; p < P; ++p) {
    for (int q = p + 1; q < P; ++q)
      if (overlap(out.p[p], no, out.p[q], no)) return MPC_E_ALIAS;
    for (const auto& in : ins) {
      if (!in.first) continue;
      for (int q = 0; q < P; ++q)
        if (in.first->p[q] && overlap(out.p[p], no, in.first->p[q], in.second)) return MPC_E_ALIAS;
    }
  }
  return MPC_OK;
}

MpIn as_in(const MpOut& o) {
  MpIn i{};
  for (int p = 0; p < kMaxParties; ++p) i.p[p] = o.p[p];
  return i;
}

}  // namespace

extern "C" {

mpc_status mpc_mp_share(mpc_ctx* c, int P, const uint64_t* x, size_t n, int src, uint64_t tag,
                        uint64_t* const* s) {
  if (!c) return MPC_E_INVAL;
  CHK(check_parties(P));
  if (src < 0 || src >= P) return MPC_E_INVAL;
  CHK(check_ptr(x, n));
  MpOut o;
  CHK(mp_out(s, P, n, &o));
  MpIn xi{};
  xi.p[0] = x;
  CHK(mp_alias(o, P, n, {{&xi, n}}));
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_mp_share(c->s[0], x, n, P, src, mp_keys(c->seed, tag, kMpShare, P), o)));
  c->stats.launches++;
  return MPC_OK;
}

mpc_status mpc_mp_reveal(mpc_ctx* c, int P, const uint64_t* const* s, size_t n, uint64_t* out) {
  if (!c) return MPC_E_INVAL;
  CHK(check_parties(P));
  MpIn in;
  CHK(mp_in(s, P, n, &in));
  CHK(check_ptr(out, n));
  for (int p = 0; p < P; ++p)
    if (overlap(out, n, in.p[p], n)) return MPC_E_ALIAS;
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_mp_reveal(c->s[0], in, P, n, out)));
  c->stats.launches++;
  c->stats.opens++;
  c->stats.open_bytes_per_party += 8 * (uint64_t)n;
  return MPC_OK;
}

mpc_status mpc_mp_dealer_triples(mpc_ctx* c, int P, mpc_triple_kind kind, uint64_t dseed, uint64_t tag,
                                 const int64_t* dims, const mpc_mp_triple* t) {
  if (!c || !dims || !t) return MPC_E_INVAL;
  CHK(check_parties(P));
  CHK(set_device(c));
  const hipStream_t st = c->s[0];
  const MpKeys ka = mp_keys(dseed, tag, kMpA, P), kb = mp_keys(dseed, tag, kMpB, P),
               kc = mp_keys(dseed, tag, kMpC, P);
  if (kind == MPC_TRIPLE_MUL || kind == MPC_TRIPLE_SQUARE) {
    if (dims[0] < 0) return MPC_E_SHAPE;
    const size_t n = (size_t)dims[0];
    const bool sq = kind == MPC_TRIPLE_SQUARE;
    MpOut a, b, cc{};
    CHK(mp_out(t->a, P, n, &a));
    CHK(mp_out(t->b, P, n, &b));
    if (!sq) CHK(mp_out(t->c, P, n, &cc));
    const MpIn bi = as_in(b), ci = as_in(cc);
    CHK(mp_alias(a, P, n, {{&bi, n}, {sq ? nullptr : &ci, n}}));
    if (!sq) CHK(mp_alias(b, P, n, {{&ci, n}}));
    if (!n) return MPC_OK;
    CHK(hip_status(launch_mp_dealer_mul(st, ka, kb, sq ? kb : kc, P, n, sq ? 1 : 0, a, b, cc)));
    c->stats.launches++;
    return end_call(c);
  }
  if (kind != MPC_TRIPLE_MATMUL) return MPC_E_UNSUPPORTED;
  const i64 M = dims[0], N = dims[1], K = dims[2];
  CHK(check_mnk(M, N, K));
  const size_t na = (size_t)(M * K), nb = (size_t)(K * N), nc = (size_t)(M * N);
  MpOut a, b, cc;
  CHK(mp_out(t->a, P, na, &a));
  CHK(mp_out(t->b, P, nb, &b));
  CHK(mp_out(t->c, P, nc, &cc));
  const MpIn bi = as_in(b), ci = as_in(cc);
  CHK(mp_alias(a, P, na, {{&bi, nb}, {&ci, nc}}));
  CHK(mp_alias(b, P, nb, {{&ci, nc}}));
  if (!na && !nb && !nc) return MPC_OK;
  const mpc_form form = resolve_form(MPC_FORM_AUTO, M, N, K, K);
  // workspace: a = sum a_p, b = sum b_p, S = sum_{p<P-1} c_p, then the GEMM's packs
  JobSpec ja = left_job(M, K, K), jb = right_job(K, N, N);
  size_t need = kAlign + align_up(na * 8) + align_up(nb * 8) + align_up(nc * 8);
  if (form == MPC_FORM_LIMB8) need += job_bytes(ja) + job_bytes(jb);
  CHK(ensure_ws(c, need));
  Carve cv(c->ws);
  u64* as = cv.take<u64>(na);
  u64* bs = cv.take<u64>(nb);
  u64* S = cv.take<u64>(nc);
  CHK(hip_status(launch_mp_fill_sum(st, ka, P, na, a, as)));
  CHK(hip_status(launch_mp_fill_sum(st, kb, P, nb, b, bs)));
  CHK(hip_status(launch_mp_fill_sum(st, kc, P - 1, nc, cc, S)));
  c->stats.launches += 3;
  if (!nc) return end_call(c);
  // c_{P-1} = a @ b - S
  const Epilogue ep = make_ep(S, -1, 0, cc.p[P - 1], rowmajor_view(N));
  if (form == MPC_FORM_LIMB8) {
    set_mode(ja, kModeCopy, {as});
    set_mode(jb, kModeCopy, {bs});
    const PackJob PA = place_job(ja, cv), PB = place_job(jb, cv);
    CHK(issue_limb(c, {PA, PB}, {limb_req(M, N, K, 0, PA.dst[0], nullptr, PB.dst[0], nullptr, ep)},
                   c->sched_default));
  } else {
    CHK(issue_plain(c, {plain_problem(M, N, K, 0, as, nullptr, K, nullptr, 0, bs, nullptr, N, nullptr, 0, ep)}));
  }
  return end_call(c);
}

mpc_status mpc_mp_dealer_trunc(mpc_ctx* c, int P, uint64_t dseed, uint64_t tag, size_t n, uint64_t* const* r,
                               uint64_t* const* theta_r) {
  if (!c) return MPC_E_INVAL;
  CHK(check_parties(P));
  MpOut ro, to;
  CHK(mp_out(r, P, n, &ro));
  CHK(mp_out(theta_r, P, n, &to));
  const MpIn ti = as_in(to);
  CHK(mp_alias(ro, P, n, {{&ti, n}}));
  CHK(mp_alias(to, P, n, {}));
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_mp_dealer_trunc(c->s[0], mp_keys(dseed, tag, kMpR, P), mp_keys(dseed, tag, kMpT, P), P,
                                        n, ro, to)));
  c->stats.launches++;
  return MPC_OK;
}

mpc_status mpc_mp_beaver_mul(mpc_ctx* c, int P, size_t n, const uint64_t* const* x, const uint64_t* const* y,
                             const mpc_mp_triple* t, uint64_t* const* z) {
  if (!c || !t) return MPC_E_INVAL;
  CHK(check_parties(P));
  const bool sq = y == nullptr;
  MpIn xi, yi{}, ai, bi, ci{};
  CHK(mp_in(x, P, n, &xi));
  if (!sq) CHK(mp_in(y, P, n, &yi));
  CHK(mp_in(t->a, P, n, &ai));
  CHK(mp_in(t->b, P, n, &bi));
  if (!sq) CHK(mp_in(t->c, P, n, &ci));
  MpOut zo;
  CHK(mp_out(z, P, n, &zo));
  CHK(mp_alias(zo, P, n, {{&xi, n}, {sq ? nullptr : &yi, n}, {&ai, n}, {&bi, n}, {sq ? nullptr : &ci, n}}));
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_mp_beaver_mul(c->s[0], xi, yi, ai, bi, ci, P, n, sq ? 1 : 0, zo)));
  c->stats.launches++;
  c->stats.opens++;
  c->stats.open_bytes_per_party += 8 * (uint64_t)n * (sq ? 1 : 2);
  return MPC_OK;
}

mpc_status mpc_mp_beaver_matmul(mpc_ctx* c, int P, int64_t M, int64_t N, int64_t K, const uint64_t* const* x,
                                const uint64_t* const* y, const mpc_mp_triple* t, mpc_form form,
                                uint64_t* const* z) {
  if (!c || !t) return MPC_E_INVAL;
  CHK(check_parties(P));
  CHK(check_form(form));
  if (form == MPC_FORM_FP64LIMB) return MPC_E_UNSUPPORTED;
  CHK(check_mnk(M, N, K));
  const size_t na = (size_t)(M * K), nb = (size_t)(K * N), nc = (size_t)(M * N);
  MpIn xi, yi, ai, bi, ci;
  CHK(mp_in(x, P, na, &xi));
  CHK(mp_in(y, P, nb, &yi));
  CHK(mp_in(t->a, P, na, &ai));
  CHK(mp_in(t->b, P, nb, &bi));
  CHK(mp_in(t->c, P, nc, &ci));
  MpOut zo;
  CHK(mp_out(z, P, nc, &zo));
  CHK(mp_alias(zo, P, nc, {{&xi, na}, {&yi, nb}, {&ai, na}, {&bi, nb}, {&ci, nc}}));
  if (!nc) return MPC_OK;
  CHK(set_device(c));
  form = resolve_form(form, M, N, 2 * K, K);
  CHK(check_limb_k(form, K));
  const hipStream_t st = c->s[0];
  // open eps (MxK) and delta (KxN) into the workspace, then party p's finish
  // z_p = c_p + [a_p + [p=0] eps | eps] @ [delta ; b_p]
  size_t need = kAlign + align_up(na * 8) + align_up(nb * 8);
  if (form == MPC_FORM_LIMB8)
    need += (size_t)(P + 1) * align_up(packed_bytes(M, K)) + (size_t)(P + 1) * align_up(packed_bytes(N, K));
  CHK(ensure_ws(c, need));
  Carve cv(c->ws);
  u64* eps = cv.take<u64>(na);
  u64* del = cv.take<u64>(nb);
  CHK(hip_status(launch_mp_open(st, xi, ai, P, na, eps)));
  CHK(hip_status(launch_mp_open(st, yi, bi, P, nb, del)));
  c->stats.launches += 2;
  if (form == MPC_FORM_LIMB8) {
    std::vector<PackJob> jobs;
    JobSpec je = left_job(M, K, K), jd = right_job(K, N, N);
    set_mode(je, kModeCopy, {eps});
    set_mode(jd, kModeCopy, {del});
    jobs.push_back(place_job(je, cv));
    jobs.push_back(place_job(jd, cv));
    std::vector<const uint8_t*> pa(P), pb(P);
    for (int p = 0; p < P; ++p) {
      JobSpec ja = left_job(M, K, K), jb = right_job(K, N, N);
      if (p == 0) set_mode(ja, kModeSum2, {ai.p[0], eps});
      else set_mode(ja, kModeCopy, {ai.p[p]});
      set_mode(jb, kModeCopy, {bi.p[p]});
      jobs.push_back(place_job(ja, cv));
      pa[p] = jobs.back().dst[0];
      jobs.push_back(place_job(jb, cv));
      pb[p] = jobs.back().dst[0];
    }
    std::vector<LimbReq> reqs;
    for (int p = 0; p < P; ++p)
      reqs.push_back(limb_req(M, N, K, K, pa[p], jobs[0].dst[0], jobs[1].dst[0], pb[p],
                              make_ep(ci.p[p], +1, 0, zo.p[p], rowmajor_view(N))));
    CHK(issue_limb(c, jobs, reqs, c->sched_default));
  } else {
    std::vector<PlainProblem> probs;
    for (int p = 0; p < P; ++p)
      probs.push_back(plain_problem(M, N, K, K, ai.p[p], p == 0 ? eps : nullptr, K, eps, K, del, nullptr, N,
                                    bi.p[p], N, make_ep(ci.p[p], +1, 0, zo.p[p], rowmajor_view(N))));
    CHK(issue_plain(c, probs));
  }
  c->stats.opens++;
  c->stats.open_bytes_per_party += 8 * (uint64_t)(na + nb);
  return end_call(c);
}

mpc_status mpc_mp_truncate(mpc_ctx* c, int P, size_t n, int bits, uint64_t* const* x, const uint64_t* const* r,
                           const uint64_t* const* theta_r) {
  if (!c) return MPC_E_INVAL;
  CHK(check_parties(P));
  if (bits < 1 || bits > 63) return MPC_E_INVAL;
  MpOut xo;
  MpIn ri, ti;
  CHK(mp_out(x, P, n, &xo));
  CHK(mp_in(r, P, n, &ri));
  CHK(mp_in(theta_r, P, n, &ti));
  CHK(mp_alias(xo, P, n, {{&ri, n}, {&ti, n}}));
  if (!n) return MPC_OK;
  CHK(set_device(c));
  CHK(hip_status(launch_mp_truncate(c->s[0], xo, ri, ti, P, n, bits)));
  c->stats.launches++;
  c->stats.opens++;
  c->stats.truncations++;
  c->stats.open_bytes_per_party += 8 * (uint64_t)n;
  return MPC_OK;
}

// ------------------------------------------------------------------ graphs
mpc_status mpc_graph_begin(mpc_ctx* c) {
  // the null stream cannot be captured
  if (!c || c->capturing || !c->s[0]) return MPC_E_INVAL;
  CHK(set_device(c));
  // finish eager work that still uses the upload slots before capturing
  CHK(sync_all(c));
  HIPCHK(hipStreamBeginCapture(c->s[0], hipStreamCaptureModeRelaxed));
  c->capturing = true;
  return MPC_OK;
}

mpc_status mpc_graph_end(mpc_ctx* c, void** graph_exec) {
  if (!c || !graph_exec || !c->capturing) return MPC_E_INVAL;
  CHK(set_device(c));
  hipGraph_t g = nullptr;
  c->capturing = false;
  std::vector<void*> allocs;
  allocs.swap(c->capture_allocs);
  auto drop = [&]() {
    for (void* p : allocs) (void)hipFree(p);
  };
  hipError_t e = hipStreamEndCapture(c->s[0], &g);
  if (e != hipSuccess) {
    drop();
    return hip_status(e);
  }
  hipGraphExec_t ge = nullptr;
  e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    drop();
    return hip_status(e);
  }
  mpc_graph* mg = new (std::nothrow) mpc_graph{ge, c, std::move(allocs)};
  if (!mg) {
    (void)hipGraphExecDestroy(ge);
    return MPC_E_NOMEM;
  }
  *graph_exec = (void*)mg;
  c->live_graphs++;
  return MPC_OK;
}

mpc_status mpc_graph_launch(mpc_ctx* c, void* graph_exec) {
  if (!c || !graph_exec) return MPC_E_INVAL;
  mpc_graph* g = (mpc_graph*)graph_exec;
  if (g->ctx != c) return MPC_E_INVAL;
  CHK(set_device(c));
  HIPCHK(hipGraphLaunch(g->exec, c->s[0]));
  return MPC_OK;
}

mpc_status mpc_graph_destroy(void* graph_exec) {
  if (!graph_exec) return MPC_OK;
  mpc_graph* g = (mpc_graph*)graph_exec;
  (void)hipSetDevice(g->ctx->device);
  // a replay still running reads the descriptor buffers
  (void)hipStreamSynchronize(g->ctx->s[0]);
  const hipError_t e = hipGraphExecDestroy(g->exec);
  for (void* p : g->allocs) (void)hipFree(p);
  g->ctx->live_graphs--;
  delete g;
  HIPCHK(e);
  return MPC_OK;
}

}  // extern "C"
