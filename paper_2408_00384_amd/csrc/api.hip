// C ABI of the tableau library: argument checks, gate encoding, launches and
// host <-> device marshalling.  Every step of the simulation itself runs in
// the kernels of gates.hip, measure_step.hip, measure_persist.hip and batch.hip.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>
#include <mutex>
#include <unordered_map>

#include "../../include/cliff.h"
#include "internal.h"

using namespace cliff;

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(CLIFF_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                  __LINE__);                                                           \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// ---------------------------------------------------------------- profiler ---
namespace cliff {

static hipEvent_t take_event(Profiler &p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Profiler::begin(int kind, hipStream_t st) {
  (void)kind;
  if (!on) return;
  open_ev = take_event(*this);
  if (open_ev) (void)hipEventRecord(open_ev, st);
}

void Profiler::end(int kind, hipStream_t st) {
  if (!on || !open_ev) return;
  hipEvent_t b = take_event(*this);
  if (!b) return;
  (void)hipEventRecord(b, st);
  pending.push_back({kind, open_ev, b});
  open_ev = nullptr;
}

hipError_t Profiler::resolve() {
  for (const Rec &r : pending) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return e;
    float ms_ = 0.f;
    e = hipEventElapsedTime(&ms_, r.a, r.b);
    if (e != hipSuccess) return e;
    ms[r.kind] += ms_;
    launches[r.kind] += 1;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
  return hipSuccess;
}

void Profiler::reset() {
  (void)resolve();
  for (int k = 0; k < kProfKinds; ++k) {
    ms[k] = 0;
    launches[k] = 0;
  }
}

Profiler::~Profiler() {
  for (const Rec &r : pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

}  // namespace cliff

struct cliff_ctx {
  Profiler prof;
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 0;
  uint64_t *dev_ops = nullptr;   // uploaded gate stream
  size_t dev_ops_cap = 0;        // words
  uint64_t *pinned = nullptr;    // pinned staging for uploads
  size_t pinned_cap = 0;         // words
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  // register-resident measurement: second stream and its events, and the
  // chunk scratch (grown on demand to the largest shape measured)
  hipStream_t aux = nullptr;
  hipEvent_t persist_ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  uint8_t *pscratch = nullptr;
  size_t pscratch_bytes = 0;
  int gate_mode = CLIFF_GATES_AUTO;
  int measure_mode = CLIFF_MEASURE_AUTO;
  uint64_t inject_abort_at = UINT64_MAX;   // test aid: see cliff_ctx_inject_abort
};

struct cliff_tab {
  bool persist_used = false;   // a register-resident pass ran (abort flag is meaningful)
  cliff_ctx *ctx = nullptr;
  Dims d{};
  Offsets o{};
  uint8_t *base = nullptr;
  TabDev dev{};
};

// ------------------------------------------------- allocation-free scratch ---
// Device memory of cliff_measure_record_noalloc: the qubit list of a pass and
// the register-resident chunk scratch live in this file-scope array, one copy
// per GPU (it belongs to the code object, loaded on each device the library
// runs on, and lives until the process ends).  Host code never uses the
// array's name as an address: the first context created on a device looks
// its address up with hipGetSymbolAddress, with that device current, and the
// entry point passes that pointer to the kernels.  Every call on a GPU shares
// the array; calls that overlap on one GPU race.
constexpr size_t kNoAllocQubitBytes = size_t(kPersistMaxWp) * 32 * 4;   // a pass: n <= 10,240 qubits (40 KB)
static_assert(kNoAllocQubitBytes % 256 == 0, "qubit area keeps the chunk scratch aligned");
static_assert(CLIFF_NOALLOC_SCRATCH_BYTES > kNoAllocQubitBytes, "scratch size");
static __device__ __align__(256) uint8_t scratch[CLIFF_NOALLOC_SCRATCH_BYTES];

static std::mutex g_noalloc_mu;
static std::unordered_map<int, uint8_t *> g_noalloc_ptr;   // device -> address of its scratch

// Called with `device` current (context creation): look up this device's
// copy of the array once.
static hipError_t noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr.count(device)) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_noalloc_ptr[device] = static_cast<uint8_t *>(ptr);
  return hipSuccess;
}

static uint8_t *noalloc_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc_ptr.find(device);
  return it == g_noalloc_ptr.end() ? nullptr : it->second;
}

extern "C" {

const char *cliff_last_error(void) { return g_err.c_str(); }

const char *cliff_strerror(int code) {
  switch (code) {
    case CLIFF_OK: return "ok";
    case CLIFF_EINVAL: return "invalid argument";
    case CLIFF_ENOMEM: return "out of memory / buffer too small";
    case CLIFF_EDEVICE: return "device (HIP) error";
    case CLIFF_EBUSY: return "busy";
    case CLIFF_EINTERNAL: return "internal consistency check failed";
    default: return "unknown error";
  }
}

int cliff_ctx_create(int device, void *hip_stream, cliff_ctx **out) {
  if (!out) return fail(CLIFF_EINVAL, "cliff_ctx_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev)
    return fail(CLIFF_EINVAL, "cliff_ctx_create: device %d out of range [0,%d)", device, ndev);
  DeviceGuard g(device);
  if (!g.ok) return fail(CLIFF_EDEVICE, "cliff_ctx_create: hipSetDevice(%d) failed", device);
  cliff_ctx *c = new (std::nothrow) cliff_ctx();
  if (!c) return fail(CLIFF_ENOMEM, "cliff_ctx_create: host allocation failed");
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete c;
    return fail(CLIFF_EDEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  }
  c->num_cus = prop.multiProcessorCount;
  e = hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
  for (hipEvent_t &ev : c->persist_ev)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) e = noalloc_setup(device);
  if (e != hipSuccess) {
    cliff_ctx_destroy(c);
    return fail(CLIFF_EDEVICE, "cliff_ctx_create: %s", hipGetErrorString(e));
  }
  *out = c;
  return CLIFF_OK;
}

int cliff_ctx_destroy(cliff_ctx *c) {
  if (!c) return CLIFF_OK;
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->aux) (void)hipStreamSynchronize(c->aux);
  if (c->dev_ops) (void)hipFree(c->dev_ops);
  if (c->pscratch) (void)hipFree(c->pscratch);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->upload_done) (void)hipEventDestroy(c->upload_done);
  if (c->aux) {
    (void)hipStreamSynchronize(c->aux);
    (void)hipStreamDestroy(c->aux);
  }
  for (hipEvent_t &e : c->persist_ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return CLIFF_OK;
}

int cliff_sync(cliff_ctx *c) {
  if (!c) return fail(CLIFF_EINVAL, "cliff_sync: NULL context");
  DeviceGuard g(c->device);
  HIP_TRY(hipStreamSynchronize(c->stream));
  return CLIFF_OK;
}

int cliff_ctx_num_cus(const cliff_ctx *c) { return c ? c->num_cus : 0; }

int cliff_calibrate(cliff_ctx *c, int kind, double *out) {
  if (!c || !out) return fail(CLIFF_EINVAL, "cliff_calibrate: NULL argument");
  if (kind != CLIFF_CAL_LDS && kind != CLIFF_CAL_VALU)
    return fail(CLIFF_EINVAL, "cliff_calibrate: kind %d (0: LDS bytes/s, 1: VALU lane ops/s)", kind);
  DeviceGuard g(c->device);
  uint32_t *sink = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  const uint32_t iters = kind == CLIFF_CAL_LDS ? 4096 : 8192;
  double work = 0;
  float ms = 0;
  hipError_t e = hipMalloc(&sink, 1024 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = launch_calibrate(kind, c->num_cus, iters, sink, c->stream, &work);   // warm-up
  if (e == hipSuccess) e = hipEventRecord(ev[0], c->stream);
  if (e == hipSuccess) e = launch_calibrate(kind, c->num_cus, iters, sink, c->stream, &work);
  if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (sink) (void)hipFree(sink);
  if (e != hipSuccess) return fail(CLIFF_EDEVICE, "cliff_calibrate: %s", hipGetErrorString(e));
  if (ms <= 0) return fail(CLIFF_EINTERNAL, "cliff_calibrate: no elapsed time");
  *out = work / (double(ms) * 1e-3);
  return CLIFF_OK;
}

int cliff_ctx_inject_abort(cliff_ctx *c, uint64_t at) {
  if (!c) return fail(CLIFF_EINVAL, "cliff_ctx_inject_abort: NULL context");
  c->inject_abort_at = at;
  return CLIFF_OK;
}

int cliff_ctx_set_measure_mode(cliff_ctx *c, int mode) {
  if (!c) return fail(CLIFF_EINVAL, "cliff_ctx_set_measure_mode: NULL context");
  if (mode < CLIFF_MEASURE_AUTO || mode > CLIFF_MEASURE_BLOCKED)
    return fail(CLIFF_EINVAL, "cliff_ctx_set_measure_mode: bad mode %d", mode);
  c->measure_mode = mode;
  return CLIFF_OK;
}

int cliff_ctx_set_gate_mode(cliff_ctx *c, int mode) {
  if (!c) return fail(CLIFF_EINVAL, "cliff_ctx_set_gate_mode: NULL context");
  if (mode < CLIFF_GATES_AUTO || mode > CLIFF_GATES_FUSED)
    return fail(CLIFF_EINVAL, "cliff_ctx_set_gate_mode: bad mode %d", mode);
  c->gate_mode = mode;
  return CLIFF_OK;
}

size_t cliff_tab_bytes(uint32_t n, uint32_t shots) {
  if (n == 0 || shots == 0 || n > kMaxQubits) return 0;
  return make_offsets(make_dims(n, shots)).total;
}

int cliff_tab_bind(cliff_ctx *ctx, uint32_t n, uint32_t shots, void *dev, size_t bytes,
                   cliff_tab **out) {
  if (!ctx || !dev || !out) return fail(CLIFF_EINVAL, "cliff_tab_bind: NULL argument");
  *out = nullptr;
  if (n == 0 || shots == 0) return fail(CLIFF_EINVAL, "cliff_tab_bind: n and shots must be > 0");
  if (n > kMaxQubits) return fail(CLIFF_EINVAL, "cliff_tab_bind: n = %u > %u", n, kMaxQubits);
  if (reinterpret_cast<uintptr_t>(dev) & 255)
    return fail(CLIFF_EINVAL, "cliff_tab_bind: device buffer not 256-byte aligned");
  const size_t need = cliff_tab_bytes(n, shots);
  if (bytes < need)
    return fail(CLIFF_ENOMEM, "cliff_tab_bind: buffer of %zu bytes < %zu needed", bytes, need);
  cliff_tab *t = new (std::nothrow) cliff_tab();
  if (!t) return fail(CLIFF_ENOMEM, "cliff_tab_bind: host allocation failed");
  t->ctx = ctx;
  t->d = make_dims(n, shots);
  t->o = make_offsets(t->d);
  t->base = reinterpret_cast<uint8_t *>(dev);
  TabDev &v = t->dev;
  auto at = [&](size_t off) { return t->base + off; };
  v.X = reinterpret_cast<uint64_t *>(at(t->o.X));
  v.Z = reinterpret_cast<uint64_t *>(at(t->o.Z));
  v.R = reinterpret_cast<uint64_t *>(at(t->o.R));
  v.P = reinterpret_cast<uint64_t *>(at(t->o.P));
  v.M = reinterpret_cast<uint64_t *>(at(t->o.M));
  v.xp = reinterpret_cast<uint64_t *>(at(t->o.xp));
  v.zp = reinterpret_cast<uint64_t *>(at(t->o.zp));
  v.rp = reinterpret_cast<uint64_t *>(at(t->o.rp));
  v.part = reinterpret_cast<uint64_t *>(at(t->o.part));
  v.state = reinterpret_cast<uint32_t *>(at(t->o.state));
  v.out = at(t->o.out);
  v.kind = at(t->o.kind);
  v.SN = reinterpret_cast<uint64_t *>(at(t->o.SN));
  v.piv = reinterpret_cast<uint32_t *>(at(t->o.piv));
  v.rps = reinterpret_cast<uint64_t *>(at(t->o.rps));
  v.detpar = reinterpret_cast<uint32_t *>(at(t->o.detpar));
  v.detY = reinterpret_cast<uint32_t *>(at(t->o.detY));
  v.detr = reinterpret_cast<uint64_t *>(at(t->o.detr));
  v.SNall = v.C1all = v.ring = v.pub = nullptr;   // chunk scratch: bound per pass
  v.pivall = nullptr;
  v.abort_flag = reinterpret_cast<uint32_t *>(at(t->o.abort_flag));
  v.n = n;
  v.S = shots;
  v.W = t->d.W;
  v.Wp = t->d.Wp;
  v.NW = t->d.NW;
  v.SW = t->d.SW;
  *out = t;
  return CLIFF_OK;
}

int cliff_tab_unbind(cliff_tab *t) {
  delete t;
  return CLIFF_OK;
}

int cliff_tab_info(const cliff_tab *t, uint32_t *n, uint32_t *shots) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_tab_info: NULL tableau");
  if (n) *n = t->d.n;
  if (shots) *shots = t->d.S;
  return CLIFF_OK;
}

int cliff_tab_init_zero(cliff_tab *t) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_tab_init_zero: NULL tableau");
  DeviceGuard g(t->ctx->device);
  HIP_TRY(launch_init_zero(t->dev, t->ctx->stream));
  return CLIFF_OK;
}

}  // extern "C"

// ------------------------------------------------------------ gate encoding ---

static int check_layers(uint32_t n, const uint8_t *h, const uint8_t *s, const uint32_t *ctrl,
                        const uint32_t *tgt, uint32_t npairs, uint32_t depth) {
  if (depth == 0) return CLIFF_OK;
  if (!h || !s) return fail(CLIFF_EINVAL, "layers: NULL h/s");
  if (npairs && (!ctrl || !tgt)) return fail(CLIFF_EINVAL, "layers: NULL ctrl/tgt");
  if (2ull * npairs > n) return fail(CLIFF_EINVAL, "layers: %u pairs on %u qubits", npairs, n);
  std::vector<uint32_t> seen(n, 0xFFFFFFFFu);
  for (uint32_t l = 0; l < depth; ++l) {
    for (uint32_t k = 0; k < npairs; ++k) {
      const uint32_t c = ctrl[size_t(l) * npairs + k], g = tgt[size_t(l) * npairs + k];
      if (c >= n || g >= n)
        return fail(CLIFF_EINVAL, "layer %u pair %u: qubit out of range (n=%u)", l, k, n);
      if (c == g) return fail(CLIFF_EINVAL, "layer %u pair %u: CNOT control == target", l, k);
      if (seen[c] == l || seen[g] == l)
        return fail(CLIFF_EINVAL, "layer %u: qubit used by two CNOTs", l);
      seen[c] = seen[g] = l;
    }
  }
  return CLIFF_OK;
}

// ops for one layer; returns the number of words written (cap permitting)
static size_t encode_layer(uint32_t n, const uint8_t *h, const uint8_t *s, const uint32_t *ctrl,
                           const uint32_t *tgt, uint32_t npairs, std::vector<uint8_t> &paired,
                           uint64_t *ops, size_t cap) {
  size_t cnt = 0;
  auto emit = [&](uint64_t v) {
    if (ops && cnt < cap) ops[cnt] = v;
    ++cnt;
  };
  static const uint32_t kHS = sq_compose(SQ_H, SQ_S);
  auto code = [&](uint32_t q) { return h[q] ? (s[q] ? kHS : SQ_H) : (s[q] ? SQ_S : SQ_I); };
  std::fill(paired.begin(), paired.end(), 0);
  for (uint32_t k = 0; k < npairs; ++k) {
    const uint32_t c = ctrl[k], g = tgt[k];
    paired[c] = paired[g] = 1;
    emit(make_op(c, g, code(c), code(g), PAIR_CNOT));
  }
  for (uint32_t q = 0; q < n; ++q) {
    if (paired[q] || !(h[q] | s[q])) continue;
    emit(make_op(q, 0, code(q), SQ_I, PAIR_NONE));
  }
  return cnt;
}

extern "C" int cliff_encode_layers(uint32_t n, const uint8_t *h, const uint8_t *s,
                                   const uint32_t *ctrl, const uint32_t *tgt, uint32_t npairs,
                                   uint32_t depth, uint64_t *ops, size_t cap, uint32_t *offs,
                                   size_t *nops) {
  if (!nops) return fail(CLIFF_EINVAL, "cliff_encode_layers: nops is NULL");
  if (n == 0) return fail(CLIFF_EINVAL, "cliff_encode_layers: n == 0");
  int rc = check_layers(n, h, s, ctrl, tgt, npairs, depth);
  if (rc) return rc;
  std::vector<uint8_t> paired(n);
  size_t total = 0;
  for (uint32_t l = 0; l < depth; ++l) {
    if (offs) offs[l] = uint32_t(total);
    const size_t room = (ops && total < cap) ? cap - total : 0;
    total += encode_layer(n, h + size_t(l) * n, s + size_t(l) * n,
                          npairs ? ctrl + size_t(l) * npairs : nullptr,
                          npairs ? tgt + size_t(l) * npairs : nullptr, npairs, paired,
                          ops ? ops + std::min(total, cap) : nullptr, room);
    if (total > 0xFFFFFFF0ull) return fail(CLIFF_EINVAL, "cliff_encode_layers: stream too long");
  }
  if (offs) offs[depth] = uint32_t(total);
  *nops = total;
  if (ops && total > cap) return fail(CLIFF_ENOMEM, "cliff_encode_layers: need %zu words", total);
  return CLIFF_OK;
}

// Staged uploads into the context's device buffer (stream-ordered): reserve
// `words` 64-bit words (waits for the previous upload's host copy, grows the
// pinned and device buffers if needed), fill the returned pinned area, then
// commit the copy.  The device base address is known before the copy, so the
// staged words may point into themselves.
static int upload_reserve(cliff_ctx *c, size_t words, uint64_t **host, uint64_t **dev) {
  if (c->upload_pending) {
    HIP_TRY(hipEventSynchronize(c->upload_done));
    c->upload_pending = false;
  }
  if (words > c->dev_ops_cap) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->dev_ops) HIP_TRY(hipFree(c->dev_ops));
    c->dev_ops = nullptr;
    c->dev_ops_cap = 0;
    size_t cap = std::max<size_t>(words, 1 << 16);
    HIP_TRY(hipMalloc(&c->dev_ops, cap * 8));
    c->dev_ops_cap = cap;
  }
  if (words > c->pinned_cap) {
    if (c->pinned) HIP_TRY(hipHostFree(c->pinned));
    c->pinned = nullptr;
    c->pinned_cap = 0;
    size_t cap = std::max<size_t>(words, 1 << 16);
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&c->pinned), cap * 8, hipHostMallocDefault));
    c->pinned_cap = cap;
  }
  *host = c->pinned;
  *dev = c->dev_ops;
  return CLIFF_OK;
}

static int upload_commit(cliff_ctx *c, size_t words) {
  HIP_TRY(hipMemcpyAsync(c->dev_ops, c->pinned, words * 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipEventRecord(c->upload_done, c->stream));
  c->upload_pending = true;
  return CLIFF_OK;
}

// Upload [ops | layer offsets]; returns device pointers to both parts.
static int upload_stream(cliff_ctx *c, const uint64_t *ops, size_t nops, const uint32_t *offs,
                         size_t noffs, const uint64_t **dev_ops, const uint32_t **dev_offs) {
  const size_t offs_words = (noffs + 1) / 2;
  const size_t words = nops + offs_words;
  if (words == 0) return CLIFF_OK;
  uint64_t *host = nullptr, *dev = nullptr;
  int rc = upload_reserve(c, words, &host, &dev);
  if (rc) return rc;
  if (nops) memcpy(host, ops, nops * 8);
  if (noffs) {
    host[nops + offs_words - 1] = 0;
    memcpy(host + nops, offs, noffs * 4);
  }
  rc = upload_commit(c, words);
  if (rc) return rc;
  if (dev_ops) *dev_ops = dev;
  if (dev_offs) *dev_offs = reinterpret_cast<const uint32_t *>(dev + nops);
  return CLIFF_OK;
}

// Run an encoded gate stream: all layers in one launch when the 32-row LDS
// slice of every column fits, otherwise one launch per layer.
static int run_encoded(cliff_tab *t, const uint64_t *dev_ops, const uint32_t *host_offs,
                       const uint32_t *dev_offs, uint32_t depth) {
  for (uint32_t l = 0; l < depth; ++l)
    if (host_offs[l + 1] < host_offs[l])
      return fail(CLIFF_EINVAL, "layer offsets decrease at layer %u", l);
  hipStream_t st = t->ctx->stream;
  const int mode = t->ctx->gate_mode;
  if (mode == CLIFF_GATES_FUSED && !(dev_offs && fused_gates_fit(t->d.n)))
    return fail(CLIFF_EINVAL, "fused gates need 8n <= %zu bytes of LDS (n = %u)", kFusedGateLds, t->d.n);
  if (mode != CLIFF_GATES_PER_LAYER && dev_offs && fused_gates_fit(t->d.n)) {
    t->ctx->prof.begin(PK_GATE, st);
    hipError_t e = launch_gates_fused(t->dev, dev_ops, dev_offs, depth, st);
    t->ctx->prof.end(PK_GATE, st);
    HIP_TRY(e);
    return CLIFF_OK;
  }
  for (uint32_t l = 0; l < depth; ++l) {
    const uint32_t a = host_offs[l], b = host_offs[l + 1];
    t->ctx->prof.begin(PK_GATE, st);
    hipError_t e = launch_gate_layer(t->dev, dev_ops + a, b - a, st);
    t->ctx->prof.end(PK_GATE, st);
    HIP_TRY(e);
  }
  return CLIFF_OK;
}

extern "C" int cliff_apply_layers(cliff_tab *t, const uint8_t *h, const uint8_t *s,
                                  const uint32_t *ctrl, const uint32_t *tgt, uint32_t npairs,
                                  uint32_t depth) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_apply_layers: NULL tableau");
  if (depth == 0) return CLIFF_OK;
  size_t nops = 0;
  std::vector<uint32_t> offs(depth + 1);
  int rc = cliff_encode_layers(t->d.n, h, s, ctrl, tgt, npairs, depth, nullptr, 0, offs.data(), &nops);
  if (rc) return rc;
  std::vector<uint64_t> ops(nops);
  rc = cliff_encode_layers(t->d.n, h, s, ctrl, tgt, npairs, depth, ops.data(), nops, offs.data(), &nops);
  if (rc) return rc;
  DeviceGuard g(t->ctx->device);
  const uint64_t *dops = nullptr;
  const uint32_t *doffs = nullptr;
  rc = upload_stream(t->ctx, ops.data(), ops.size(), offs.data(), offs.size(), &dops, &doffs);
  if (rc) return rc;
  return run_encoded(t, dops, offs.data(), doffs, depth);
}

extern "C" int cliff_apply_encoded(cliff_tab *t, const uint64_t *dev_ops, const uint32_t *offs,
                                   uint32_t depth) {
  if (!t || !offs || (!dev_ops && depth)) return fail(CLIFF_EINVAL, "cliff_apply_encoded: NULL argument");
  if (depth == 0) return CLIFF_OK;
  DeviceGuard g(t->ctx->device);
  const uint32_t *doffs = nullptr;
  if (fused_gates_fit(t->d.n) && t->ctx->gate_mode != CLIFF_GATES_PER_LAYER) {
    int rc = upload_stream(t->ctx, nullptr, 0, offs, size_t(depth) + 1, nullptr, &doffs);
    if (rc) return rc;
  }
  return run_encoded(t, dev_ops, offs, doffs, depth);
}

// Gate list -> encoded layers.  Greedy layering: a gate joins the current
// layer unless it would have to act after an op of that layer on one of its
// qubits.  A single-qubit gate on a qubit that only single-qubit gates of the
// layer touched is composed into that op's code; a two-qubit gate takes over
// the pending single-qubit codes of its qubits as its "before" parts.  Ops of
// a layer act on disjoint qubits and commute exactly, and the order of the
// list is kept on every qubit.
static int encode_gate_list(uint32_t n, const uint8_t *op, const uint32_t *a, const uint32_t *b,
                            size_t count, std::vector<uint64_t> &ops, std::vector<uint32_t> &offs) {
  static const uint32_t kCode[7] = {SQ_H, SQ_S, 0, SQ_SDG, SQ_X, SQ_Y, SQ_Z};
  for (size_t k = 0; k < count; ++k) {
    if (op[k] > CLIFF_OP_SWAP) return fail(CLIFF_EINVAL, "gate %zu: bad op %u", k, op[k]);
    if (a[k] >= n) return fail(CLIFF_EINVAL, "gate %zu: qubit %u >= n = %u", k, a[k], n);
    const bool two = op[k] == CLIFF_OP_CNOT || op[k] == CLIFF_OP_CZ || op[k] == CLIFF_OP_SWAP;
    if (two) {
      if (b[k] >= n) return fail(CLIFF_EINVAL, "gate %zu: second qubit %u >= n = %u", k, b[k], n);
      if (a[k] == b[k]) return fail(CLIFF_EINVAL, "gate %zu: two-qubit gate on one qubit", k);
    }
  }
  // per qubit: the layer that last touched it, and the slot of its op there
  // (slot_pair marks a two-qubit op, after which nothing may join the qubit)
  std::vector<uint32_t> layer_of(n, 0), slot(n, 0);
  std::vector<uint8_t> slot_pair(n, 0);
  std::vector<uint64_t> cur;          // ops of the current layer
  std::vector<uint8_t> gone;          // 1 = taken over by a later two-qubit op
  uint32_t layer = 1;
  ops.clear();
  offs.assign(1, 0);
  auto flush = [&]() {
    // single-qubit ops that composed to the identity are dropped here
    for (size_t i = 0; i < cur.size(); ++i)
      if (!gone[i] && (op_pair(cur[i]) != PAIR_NONE || op_ca(cur[i]) != SQ_I)) ops.push_back(cur[i]);
    cur.clear();
    gone.clear();
    offs.push_back(uint32_t(ops.size()));
    ++layer;
  };
  for (size_t k = 0; k < count; ++k) {
    const uint32_t qa = a[k];
    if (op[k] == CLIFF_OP_CNOT || op[k] == CLIFF_OP_CZ || op[k] == CLIFF_OP_SWAP) {
      const uint32_t qb = b[k];
      if ((layer_of[qa] == layer && slot_pair[qa]) || (layer_of[qb] == layer && slot_pair[qb])) flush();
      uint32_t ca = SQ_I, cb = SQ_I;
      if (layer_of[qa] == layer) { ca = op_ca(cur[slot[qa]]); gone[slot[qa]] = 1; }
      if (layer_of[qb] == layer) { cb = op_ca(cur[slot[qb]]); gone[slot[qb]] = 1; }
      const uint32_t pair = op[k] == CLIFF_OP_CNOT ? PAIR_CNOT : op[k] == CLIFF_OP_CZ ? PAIR_CZ : PAIR_SWAP;
      layer_of[qa] = layer_of[qb] = layer;
      slot[qa] = slot[qb] = uint32_t(cur.size());
      slot_pair[qa] = slot_pair[qb] = 1;
      cur.push_back(make_op(qa, qb, ca, cb, pair));
      gone.push_back(0);
    } else {
      const uint32_t g = kCode[op[k]];
      if (layer_of[qa] == layer && slot_pair[qa]) flush();
      if (layer_of[qa] == layer) {
        uint64_t &v = cur[slot[qa]];
        v = make_op(qa, 0, sq_compose(op_ca(v), g), SQ_I, PAIR_NONE);
      } else {
        layer_of[qa] = layer;
        slot[qa] = uint32_t(cur.size());
        slot_pair[qa] = 0;
        cur.push_back(make_op(qa, 0, g, SQ_I, PAIR_NONE));
        gone.push_back(0);
      }
    }
    if (ops.size() + cur.size() > 0xFFFFFFF0ull) return fail(CLIFF_EINVAL, "gate list too long");
  }
  if (!cur.empty()) flush();
  return CLIFF_OK;
}

extern "C" int cliff_apply_gates(cliff_tab *t, const uint8_t *op, const uint32_t *a,
                                 const uint32_t *b, size_t count) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_apply_gates: NULL tableau");
  if (count == 0) return CLIFF_OK;
  if (!op || !a || !b) return fail(CLIFF_EINVAL, "cliff_apply_gates: NULL array");
  const uint32_t n = t->d.n;
  std::vector<uint64_t> ops;
  std::vector<uint32_t> offs;
  int rc = encode_gate_list(n, op, a, b, count, ops, offs);
  if (rc) return rc;
  if (ops.empty()) return CLIFF_OK;   // every gate cancelled out
  DeviceGuard g(t->ctx->device);
  const uint64_t *dops = nullptr;
  const uint32_t *doffs = nullptr;
  rc = upload_stream(t->ctx, ops.data(), ops.size(), offs.data(), offs.size(), &dops, &doffs);
  if (rc) return rc;
  return run_encoded(t, dops, offs.data(), doffs, uint32_t(offs.size() - 1));
}

// --------------------------------------------------------- many tableaux ---

extern "C" int cliff_encode_gates(uint32_t n, const uint8_t *op, const uint32_t *a, const uint32_t *b,
                                  size_t count, uint64_t *ops, size_t ops_cap, uint32_t *offs,
                                  size_t offs_cap, size_t *nops, uint32_t *depth) {
  if (!nops || !depth) return fail(CLIFF_EINVAL, "cliff_encode_gates: nops/depth is NULL");
  if (n == 0) return fail(CLIFF_EINVAL, "cliff_encode_gates: n == 0");
  if (count && (!op || !a || !b)) return fail(CLIFF_EINVAL, "cliff_encode_gates: NULL array");
  std::vector<uint64_t> v;
  std::vector<uint32_t> o;
  int rc = encode_gate_list(n, op, a, b, count, v, o);
  if (rc) return rc;
  *nops = v.size();
  *depth = uint32_t(o.size() - 1);
  if (ops && v.size() > ops_cap) return fail(CLIFF_ENOMEM, "cliff_encode_gates: need %zu op words", v.size());
  if (offs && o.size() > offs_cap) return fail(CLIFF_ENOMEM, "cliff_encode_gates: need %zu offsets", o.size());
  if (ops) memcpy(ops, v.data(), v.size() * 8);
  if (offs) memcpy(offs, o.data(), o.size() * 4);
  return CLIFF_OK;
}

// One tableau's part of a many-tableau launch: ops staged from the host
// (host_ops) or already on the device (dev_ops), and host layer offsets.
struct ManySource {
  const uint64_t *host_ops = nullptr;
  size_t nops = 0;
  const uint64_t *dev_ops = nullptr;
  const uint32_t *offs = nullptr;
  uint32_t depth = 0;
};

// Descriptors, staged ops and every tableau's offsets in one upload; one launch.
static int run_many(cliff_tab *const *tabs, const std::vector<ManySource> &src, int rows_per_group) {
  const size_t count = src.size();
  if (count == 0) return CLIFF_OK;
  if (count > 65535) return fail(CLIFF_EINVAL, "many-tableau gates: %zu tableaux > 65535", count);
  if (!tabs) return fail(CLIFF_EINVAL, "many-tableau gates: NULL tableau array");
  cliff_ctx *c = tabs[0] ? tabs[0]->ctx : nullptr;
  uint32_t max_n = 0;
  size_t groups64 = 0;
  for (size_t i = 0; i < count; ++i) {
    if (!tabs[i]) return fail(CLIFF_EINVAL, "many-tableau gates: tableau %zu is NULL", i);
    if (tabs[i]->ctx != c) return fail(CLIFF_EINVAL, "many-tableau gates: tableaux on different contexts");
    if (src[i].depth && !src[i].offs) return fail(CLIFF_EINVAL, "many-tableau gates: NULL offsets (%zu)", i);
    for (uint32_t l = 0; l < src[i].depth; ++l)
      if (src[i].offs[l + 1] < src[i].offs[l])
        return fail(CLIFF_EINVAL, "tableau %zu: layer offsets decrease at layer %u", i, l);
    if (src[i].depth && src[i].offs[src[i].depth] && !src[i].host_ops && !src[i].dev_ops)
      return fail(CLIFF_EINVAL, "many-tableau gates: NULL ops (%zu)", i);
    max_n = std::max(max_n, tabs[i]->d.n);
    groups64 += tabs[i]->d.W;
  }
  {
    std::vector<const cliff_tab *> sorted(tabs, tabs + count);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(CLIFF_EINVAL, "many-tableau gates: a tableau appears twice");
  }
  uint32_t rows;
  if (rows_per_group == 0)
    rows = (many_gates_fit(max_n, 64) && groups64 >= 4 * size_t(c->num_cus)) ? 64 : 32;
  else if (rows_per_group == 32 || rows_per_group == 64 || rows_per_group == 128)
    rows = uint32_t(rows_per_group);
  else
    return fail(CLIFF_EINVAL, "rows_per_group must be 0, 32, 64 or 128 (got %d)", rows_per_group);
  if (!many_gates_fit(max_n, rows))
    return fail(CLIFF_EINVAL, "many-tableau gates: n = %u does not fit LDS at %u rows per group", max_n, rows);
  const size_t desc_words = count * (sizeof(ManyDesc) / 8);
  size_t words = desc_words;
  for (const ManySource &m : src) words += (m.host_ops ? m.nops : 0) + (size_t(m.depth) + 2) / 2;
  DeviceGuard g(c->device);
  uint64_t *host = nullptr, *dev = nullptr;
  int rc = upload_reserve(c, words, &host, &dev);
  if (rc) return rc;
  ManyDesc *hd = reinterpret_cast<ManyDesc *>(host);
  size_t at = desc_words;
  for (size_t i = 0; i < count; ++i) {
    const ManySource &m = src[i];
    ManyDesc d{};
    d.X = tabs[i]->dev.X;
    d.Z = tabs[i]->dev.Z;
    d.P = tabs[i]->dev.P;
    d.n = tabs[i]->d.n;
    d.Wp = tabs[i]->d.Wp;
    d.depth = m.depth;
    if (m.host_ops) {
      if (m.nops) memcpy(host + at, m.host_ops, m.nops * 8);
      d.ops = dev + at;
      at += m.nops;
    } else {
      d.ops = m.dev_ops;
    }
    const size_t ow = (size_t(m.depth) + 2) / 2;
    host[at + ow - 1] = 0;
    if (m.depth) memcpy(host + at, m.offs, (size_t(m.depth) + 1) * 4);
    else reinterpret_cast<uint32_t *>(host + at)[0] = 0;
    d.offs = reinterpret_cast<const uint32_t *>(dev + at);
    at += ow;
    hd[i] = d;
  }
  rc = upload_commit(c, words);
  if (rc) return rc;
  c->prof.begin(PK_GATE, c->stream);
  hipError_t e = launch_gates_many(reinterpret_cast<const ManyDesc *>(dev), uint32_t(count), max_n, rows,
                                   c->stream);
  c->prof.end(PK_GATE, c->stream);
  HIP_TRY(e);
  return CLIFF_OK;
}

extern "C" int cliff_apply_encoded_many(cliff_tab *const *tabs, const uint64_t *const *dev_ops,
                                        const uint32_t *const *offs, const uint32_t *depths, size_t count,
                                        int rows_per_group) {
  if (count == 0) return CLIFF_OK;
  if (!dev_ops || !offs || !depths) return fail(CLIFF_EINVAL, "cliff_apply_encoded_many: NULL array");
  std::vector<ManySource> src(count);
  for (size_t i = 0; i < count; ++i) {
    src[i].dev_ops = dev_ops[i];
    src[i].offs = offs[i];
    src[i].depth = depths[i];
  }
  return run_many(tabs, src, rows_per_group);
}

extern "C" int cliff_apply_gates_many(cliff_tab *const *tabs, const uint8_t *const *op,
                                      const uint32_t *const *a, const uint32_t *const *b,
                                      const size_t *counts, size_t count, int rows_per_group) {
  if (count == 0) return CLIFF_OK;
  if (!tabs || !op || !a || !b || !counts) return fail(CLIFF_EINVAL, "cliff_apply_gates_many: NULL array");
  std::vector<std::vector<uint64_t>> ops(count);
  std::vector<std::vector<uint32_t>> offs(count);
  std::vector<ManySource> src(count);
  for (size_t i = 0; i < count; ++i) {
    if (!tabs[i]) return fail(CLIFF_EINVAL, "cliff_apply_gates_many: tableau %zu is NULL", i);
    if (counts[i] && (!op[i] || !a[i] || !b[i])) return fail(CLIFF_EINVAL, "cliff_apply_gates_many: NULL list %zu", i);
    int rc = encode_gate_list(tabs[i]->d.n, op[i], a[i], b[i], counts[i], ops[i], offs[i]);
    if (rc) return rc;
    src[i].host_ops = ops[i].data();
    src[i].nops = ops[i].size();
    src[i].offs = offs[i].data();
    src[i].depth = uint32_t(offs[i].size() - 1);
  }
  return run_many(tabs, src, rows_per_group);
}

// ---------------------------------------------------------------- measure ---

// One pass of up to n measurements: the register-resident path when the
// tableau shape allows it (and the device takes the cooperative launch),
// else one step kernel per measurement.
// `abort_at` (test aid): the pass's measurement at which its workgroups give
// up as on a timed-out wait, or UINT64_MAX.
// The context's chunk scratch (`need` bytes: the per-measurement kernels'
// and, when used, the blocked pass's), grown (after both streams drain) when
// a larger shape comes along.
static int ctx_persist_scratch(cliff_ctx *c, size_t need, uint8_t **base) {
  if (c->pscratch_bytes < need) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipStreamSynchronize(c->aux));
    if (c->pscratch) HIP_TRY(hipFree(c->pscratch));
    c->pscratch = nullptr;
    c->pscratch_bytes = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&c->pscratch), need);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(CLIFF_ENOMEM, "measurement scratch of %zu bytes: %s", need, hipGetErrorString(e));
    }
    c->pscratch_bytes = need;
  }
  *base = c->pscratch;
  return CLIFF_OK;
}

static int noalloc_persist_scratch(cliff_ctx *c, const Dims &d, const uint32_t *qubits, size_t cnt,
                                   uint32_t *kc, uint8_t **base, const uint32_t **dev_qubits);

// `noalloc`: the chunk scratch and qubit list come from the static array and
// nothing is allocated (cliff_measure_record_noalloc).
static int measure_pass(cliff_tab *t, const uint32_t *qubits, size_t cnt, uint64_t seed,
                        uint64_t circuit, uint64_t shot0, uint64_t m0, uint64_t abort_at, bool noalloc) {
  cliff_ctx *c = t->ctx;
  hipStream_t st = c->stream;
  uint32_t G, L, CW;
  const bool shape_ok = persist_layout(t->d.n) && persist_shape(t->d.n, uint32_t(c->num_cus), &G, &L, &CW);
  uint32_t bG = 0, bL = 0;
  const bool blk_ok = shape_ok && blk_shape(t->d.n, uint32_t(c->num_cus), &bG, &bL);
  if ((c->measure_mode == CLIFF_MEASURE_PERSISTENT || c->measure_mode == CLIFF_MEASURE_BLOCKED) && !shape_ok)
    return fail(CLIFF_EINVAL, "register-resident measurement does not fit n = %u", t->d.n);
  // the allocation-free entry keeps to the per-measurement kernels
  const bool use_blk = !noalloc && blk_ok &&
                       (c->measure_mode == CLIFF_MEASURE_BLOCKED ||
                        (c->measure_mode == CLIFF_MEASURE_AUTO && t->d.n >= kBlkAutoMinN));
  if (c->measure_mode != CLIFF_MEASURE_STEP && shape_ok) {
    const uint32_t *dq = nullptr;
    uint8_t *base = nullptr;
    uint32_t kc = 0;
    int rc;
    size_t blk_at = 0, blk_set = 0;
    if (noalloc) {
      rc = noalloc_persist_scratch(c, t->d, qubits, cnt, &kc, &base, &dq);
    } else {
      auto need_for = [&](uint32_t kc_) {
        size_t need = persist_scratch_layout(t->d, kc_).total;
        if (use_blk) {
          blk_at = align256(need);
          blk_set = align256(blk_scratch_layout(t->d, kc_, bG).total);
          need = blk_at + 2 * blk_set;
        }
        return need;
      };
      kc = persist_chunk(t->d.n, use_blk);
      rc = upload_stream(c, nullptr, 0, qubits, cnt, nullptr, &dq);
      if (!rc) {
        rc = ctx_persist_scratch(c, need_for(kc), &base);
        // the blocked pass's large chunks did not fit in device memory: the
        // per-measurement path's chunk size (same results, more chunks)
        const uint32_t kc_small = persist_chunk(t->d.n, false);
        if (rc == CLIFF_ENOMEM && kc_small < kc) {
          kc = kc_small;
          rc = ctx_persist_scratch(c, need_for(kc), &base);
        }
      }
    }
    if (rc) return rc;
    TabDev dv = t->dev;
    persist_scratch_bind(dv, t->d, kc, base);
    BlkDev bsets[2];
    if (use_blk)
      for (int i = 0; i < 2; ++i) bsets[i] = blk_scratch_bind(t->d, kc, bG, base + blk_at + size_t(i) * blk_set);
    PersistStreams ps{st, c->aux, {c->persist_ev[0], c->persist_ev[1], c->persist_ev[2], c->persist_ev[3],
                                   c->persist_ev[4], c->persist_ev[5]}};
    uint32_t done = 0;
    hipError_t e = launch_measure_persist(dv, kc, dq, uint32_t(cnt), seed, circuit, shot0, m0,
                                          c->num_cus, ps, &c->prof, &done, abort_at,
                                          use_blk ? bsets : nullptr, bG, bL);
    if (done) t->persist_used = true;
    if (e == hipSuccess) return CLIFF_OK;
    (void)hipGetLastError();
    if (c->measure_mode == CLIFF_MEASURE_PERSISTENT || c->measure_mode == CLIFF_MEASURE_BLOCKED || done)
      return fail(CLIFF_EDEVICE, "cooperative launch failed after %u measurements: %s", done,
                  hipGetErrorString(e));
    // nothing measured yet: fall through, the step kernels need no co-residency
  }
  HIP_TRY(launch_measure_list(t->dev, qubits, uint32_t(cnt), seed, circuit, shot0, m0, st, &c->prof));
  return CLIFF_OK;
}

// A register-resident pass that gave up (a wait timed out) leaves the abort
// flag raised; it stays raised -- later chunks skip their work -- until a
// synchronizing call reports it here, which lowers it again.
static int check_abort(cliff_tab *t) {
  if (!t->persist_used) return CLIFF_OK;
  uint32_t v = 0;
  HIP_TRY(hipMemcpyAsync(&v, t->dev.abort_flag, 4, hipMemcpyDeviceToHost, t->ctx->stream));
  HIP_TRY(hipStreamSynchronize(t->ctx->stream));
  if (v) {
    const uint32_t zero = 0;
    HIP_TRY(hipMemcpyAsync(t->dev.abort_flag, &zero, 4, hipMemcpyHostToDevice, t->ctx->stream));
    HIP_TRY(hipStreamSynchronize(t->ctx->stream));
    return fail(CLIFF_EINTERNAL, "register-resident measurement gave up waiting for a peer workgroup; "
                                 "the tableau's contents are undefined");
  }
  return CLIFF_OK;
}

// Where a measurement call's outcomes go besides the device staging: a
// caller-owned device record, rec[s * ld + col0 + i] (shot s, measurement
// i), and random flags rnd[col0 + i] (nullable).
struct DevRecord {
  uint8_t *rec = nullptr;
  size_t ld = 0, col0 = 0;
  uint8_t *rnd = nullptr;
};

// Outcome of measurement i of shot s lands at host_out[s * ld + col0 + i].
static int measure_impl(cliff_tab *t, const uint32_t *qubits, size_t k, uint64_t seed,
                        uint64_t circuit, uint64_t shot0, uint64_t m0, uint8_t *host_out,
                        uint8_t *host_random, size_t ld, size_t col0, const DevRecord *dr = nullptr,
                        bool noalloc = false) {
  const uint32_t n = t->d.n, S = t->d.S;
  for (size_t i = 0; i < k; ++i)
    if (qubits[i] >= n) return fail(CLIFF_EINVAL, "measure: qubit %u >= n = %u", qubits[i], n);
  hipStream_t st = t->ctx->stream;
  t->ctx->prof.begin(PK_OTHER, st);
  hipError_t fe = launch_fold_pending(t->dev, st);
  t->ctx->prof.end(PK_OTHER, st);
  HIP_TRY(fe);
  std::vector<uint8_t> out_stage, kind_stage;
  // a pending injection counts down over the context's measurements
  const uint64_t inject = t->ctx->inject_abort_at;
  if (inject != UINT64_MAX) t->ctx->inject_abort_at = inject >= k ? inject - k : UINT64_MAX;
  for (size_t base = 0; base < k; base += n) {
    const size_t cnt = std::min<size_t>(n, k - base);
    const uint64_t at = (inject != UINT64_MAX && inject >= base && inject - base < cnt) ? inject - base : UINT64_MAX;
    int rc = measure_pass(t, qubits + base, cnt, seed, circuit, shot0, m0 + base, at, noalloc);
    if (rc) return rc;
    if (dr && dr->rec) {
      t->ctx->prof.begin(PK_OTHER, st);
      hipError_t e = launch_record(t->dev, uint32_t(cnt), dr->rec, dr->ld, dr->col0 + base, dr->rnd, st);
      t->ctx->prof.end(PK_OTHER, st);
      HIP_TRY(e);
    }
    if (host_out || host_random) {
      out_stage.resize(cnt * S);
      kind_stage.resize(cnt);
      HIP_TRY(hipMemcpyAsync(out_stage.data(), t->dev.out, cnt * S, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(kind_stage.data(), t->dev.kind, cnt, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      int arc = check_abort(t);
      if (arc) return arc;
      if (host_out)
        for (size_t i = 0; i < cnt; ++i)
          for (uint32_t s = 0; s < S; ++s) host_out[size_t(s) * ld + col0 + base + i] = out_stage[i * S + s];
      if (host_random) memcpy(host_random + col0 + base, kind_stage.data(), cnt);
    }
  }
  return CLIFF_OK;
}

extern "C" int cliff_measure(cliff_tab *t, const uint32_t *qubits, size_t k, uint64_t seed,
                             uint64_t circuit, uint64_t shot0, uint64_t m0, uint8_t *host_out,
                             uint8_t *host_random) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_measure: NULL tableau");
  if (k == 0) return CLIFF_OK;
  if (!qubits) return fail(CLIFF_EINVAL, "cliff_measure: NULL qubits");
  DeviceGuard g(t->ctx->device);
  return measure_impl(t, qubits, k, seed, circuit, shot0, m0, host_out, host_random, k, 0);
}

// One layer of single-qubit ops (distinct qubits), uploaded and applied.
static int apply_one_layer(cliff_tab *t, const std::vector<uint64_t> &ops) {
  if (ops.empty()) return CLIFF_OK;
  const uint32_t offs[2] = {0, uint32_t(ops.size())};
  const uint64_t *dops = nullptr;
  const uint32_t *doffs = nullptr;
  int rc = upload_stream(t->ctx, ops.data(), ops.size(), offs, 2, &dops, &doffs);
  if (rc) return rc;
  return run_encoded(t, dops, offs, doffs, 1);
}

extern "C" int cliff_measure_bases(cliff_tab *t, const uint32_t *qubits, const uint8_t *bases,
                                   size_t k, uint64_t seed, uint64_t circuit, uint64_t shot0,
                                   uint64_t m0, uint8_t *host_out, uint8_t *host_random) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_measure_bases: NULL tableau");
  if (k == 0) return CLIFF_OK;
  if (!qubits || !bases) return fail(CLIFF_EINVAL, "cliff_measure_bases: NULL qubits/bases");
  const uint32_t n = t->d.n;
  for (size_t i = 0; i < k; ++i) {
    if (qubits[i] >= n) return fail(CLIFF_EINVAL, "measure: qubit %u >= n = %u", qubits[i], n);
    if (bases[i] > CLIFF_BASIS_Y) return fail(CLIFF_EINVAL, "measure: bad basis %u at %zu", bases[i], i);
  }
  DeviceGuard g(t->ctx->device);
  // U maps the measured Pauli to Z: X -> H; Y -> S^dagger then H.  U^-1:
  // H; H then S.
  static const uint32_t kToZ[3] = {SQ_I, SQ_H, sq_compose(SQ_SDG, SQ_H)};
  static const uint32_t kBack[3] = {SQ_I, SQ_H, sq_compose(SQ_H, SQ_S)};
  std::vector<uint32_t> seen(n, 0);
  std::vector<uint64_t> pre, post;
  uint32_t run = 0;
  for (size_t i = 0; i < k;) {
    ++run;
    pre.clear();
    post.clear();
    size_t j = i;
    for (; j < k && seen[qubits[j]] != run; ++j) {
      seen[qubits[j]] = run;
      if (bases[j] != CLIFF_BASIS_Z) {
        pre.push_back(make_op(qubits[j], 0, kToZ[bases[j]], SQ_I, PAIR_NONE));
        post.push_back(make_op(qubits[j], 0, kBack[bases[j]], SQ_I, PAIR_NONE));
      }
    }
    int rc = apply_one_layer(t, pre);
    if (!rc) rc = measure_impl(t, qubits + i, j - i, seed, circuit, shot0, m0 + i, host_out, host_random, k, i);
    if (!rc) rc = apply_one_layer(t, post);
    if (rc) return rc;
    i = j;
  }
  return CLIFF_OK;
}

extern "C" int cliff_measure_record(cliff_tab *t, const uint32_t *qubits, size_t k, uint64_t seed,
                                    uint64_t circuit, uint64_t shot0, uint64_t m0, uint8_t *dev_record,
                                    size_t ld, size_t col0, uint8_t *dev_random) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_measure_record: NULL tableau");
  if (k == 0) return CLIFF_OK;
  if (!qubits || !dev_record) return fail(CLIFF_EINVAL, "cliff_measure_record: NULL qubits/record");
  if (col0 + k > ld) return fail(CLIFF_EINVAL, "cliff_measure_record: columns %zu..%zu beyond ld = %zu", col0, col0 + k, ld);
  DeviceGuard g(t->ctx->device);
  DevRecord dr{dev_record, ld, col0, dev_random};
  return measure_impl(t, qubits, k, seed, circuit, shot0, m0, nullptr, nullptr, k, 0, &dr);
}

// Chunk scratch and qubit list of a register-resident pass in the static
// array: the qubits go there through kernel arguments (no staging buffer, no
// copy from pageable memory), and the chunk is as large as fits.
static int noalloc_persist_scratch(cliff_ctx *c, const Dims &d, const uint32_t *qubits, size_t cnt,
                                   uint32_t *kc, uint8_t **base, const uint32_t **dev_qubits) {
  uint8_t *sp = noalloc_ptr(c->device);
  if (!sp) return fail(CLIFF_EINTERNAL, "no static scratch looked up for device %d", c->device);
  if (cnt * 4 > kNoAllocQubitBytes)
    return fail(CLIFF_EINVAL, "noalloc: %zu measurements in one pass exceed the %zu-byte qubit area", cnt,
                kNoAllocQubitBytes);
  const size_t room = CLIFF_NOALLOC_SCRATCH_BYTES - kNoAllocQubitBytes;
  uint32_t k = persist_chunk(d.n);
  while (k > 1 && persist_scratch_layout(d, k).total > room) k = std::max<uint32_t>(1, k * 3 / 4);
  if (persist_scratch_layout(d, k).total > room)
    return fail(CLIFF_ENOMEM, "noalloc: chunk scratch of n = %u needs %zu bytes, the static array holds %zu",
                d.n, persist_scratch_layout(d, 1).total, room);
  uint32_t *dq = reinterpret_cast<uint32_t *>(sp);
  HIP_TRY(launch_store_words(dq, qubits, uint32_t(cnt), c->stream));
  *kc = k;
  *base = sp + kNoAllocQubitBytes;
  *dev_qubits = dq;
  return CLIFF_OK;
}

extern "C" int cliff_measure_record_noalloc(cliff_tab *t, const uint32_t *qubits, size_t k, uint64_t seed,
                                            uint64_t circuit, uint64_t shot0, uint64_t m0, uint8_t *dev_record,
                                            size_t ld, size_t col0, uint8_t *dev_random) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_measure_record_noalloc: NULL tableau");
  if (k == 0) return CLIFF_OK;
  if (!qubits || !dev_record) return fail(CLIFF_EINVAL, "cliff_measure_record_noalloc: NULL qubits/record");
  if (col0 + k > ld)
    return fail(CLIFF_EINVAL, "cliff_measure_record_noalloc: columns %zu..%zu beyond ld = %zu", col0, col0 + k, ld);
  if (t->ctx->prof.on) return fail(CLIFF_EINVAL, "cliff_measure_record_noalloc: kernel timing is on (it allocates events)");
  DeviceGuard g(t->ctx->device);
  DevRecord dr{dev_record, ld, col0, dev_random};
  return measure_impl(t, qubits, k, seed, circuit, shot0, m0, nullptr, nullptr, k, 0, &dr, true);
}

// Conditional Paulis staged as op words (qubit | Pauli << 24 | column << 32).
static int cond_paulis(cliff_tab *t, const std::vector<uint64_t> &ops, const uint8_t *rec, size_t ld) {
  if (ops.empty()) return CLIFF_OK;
  const uint64_t *dops = nullptr;
  int rc = upload_stream(t->ctx, ops.data(), ops.size(), nullptr, 0, &dops, nullptr);
  if (rc) return rc;
  hipStream_t st = t->ctx->stream;
  t->ctx->prof.begin(PK_GATE, st);
  hipError_t e = launch_cond_pauli(t->dev, dops, uint32_t(ops.size()), rec, ld, st);
  t->ctx->prof.end(PK_GATE, st);
  HIP_TRY(e);
  return CLIFF_OK;
}

extern "C" int cliff_apply_cond_paulis(cliff_tab *t, const uint32_t *qubits, const uint8_t *paulis,
                                       const uint32_t *cols, size_t k, const uint8_t *dev_record, size_t ld) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_apply_cond_paulis: NULL tableau");
  if (k == 0) return CLIFF_OK;
  if (!qubits || !paulis || !cols || !dev_record) return fail(CLIFF_EINVAL, "cliff_apply_cond_paulis: NULL array");
  if (k > 0xFFFFFFFFull) return fail(CLIFF_EINVAL, "cliff_apply_cond_paulis: too many ops");
  std::vector<uint64_t> ops(k);
  for (size_t i = 0; i < k; ++i) {
    if (qubits[i] >= t->d.n) return fail(CLIFF_EINVAL, "conditional Pauli %zu: qubit %u >= n = %u", i, qubits[i], t->d.n);
    if (paulis[i] < 1 || paulis[i] > 3) return fail(CLIFF_EINVAL, "conditional Pauli %zu: bad Pauli %u", i, paulis[i]);
    if (cols[i] >= ld) return fail(CLIFF_EINVAL, "conditional Pauli %zu: column %u >= ld = %zu", i, cols[i], ld);
    ops[i] = uint64_t(qubits[i]) | (uint64_t(paulis[i]) << 24) | (uint64_t(cols[i]) << 32);
  }
  DeviceGuard g(t->ctx->device);
  return cond_paulis(t, ops, dev_record, ld);
}

extern "C" int cliff_reset_record(cliff_tab *t, const uint32_t *qubits, size_t k, uint64_t seed,
                                  uint64_t circuit, uint64_t shot0, uint64_t m0, uint8_t *dev_record,
                                  size_t ld, size_t col0, uint8_t *dev_random) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_reset_record: NULL tableau");
  if (k == 0) return CLIFF_OK;
  if (!qubits || !dev_record) return fail(CLIFF_EINVAL, "cliff_reset_record: NULL qubits/record");
  if (col0 + k > ld) return fail(CLIFF_EINVAL, "cliff_reset_record: columns %zu..%zu beyond ld = %zu", col0, col0 + k, ld);
  const uint32_t n = t->d.n;
  for (size_t i = 0; i < k; ++i)
    if (qubits[i] >= n) return fail(CLIFF_EINVAL, "reset: qubit %u >= n = %u", qubits[i], n);
  DeviceGuard g(t->ctx->device);
  // per run of distinct qubits: measure them all, then X in the shots whose
  // outcome was 1 (a repeated qubit must see its earlier reset first)
  std::vector<uint32_t> seen(n, 0);
  std::vector<uint64_t> xs;
  uint32_t run = 0;
  for (size_t i = 0; i < k;) {
    ++run;
    size_t j = i;
    for (; j < k && seen[qubits[j]] != run; ++j) seen[qubits[j]] = run;
    DevRecord dr{dev_record, ld, col0 + i, dev_random};
    int rc = measure_impl(t, qubits + i, j - i, seed, circuit, shot0, m0 + i, nullptr, nullptr, k, 0, &dr);
    if (rc) return rc;
    xs.clear();
    for (size_t q = i; q < j; ++q) xs.push_back(uint64_t(qubits[q]) | (1ull << 24) | (uint64_t(col0 + q) << 32));
    rc = cond_paulis(t, xs, dev_record, ld);
    if (rc) return rc;
    i = j;
  }
  return CLIFF_OK;
}

extern "C" int cliff_measure_async(cliff_tab *t, const uint32_t *qubits, size_t k, uint64_t seed,
                                   uint64_t circuit, uint64_t shot0, uint64_t m0) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_measure_async: NULL tableau");
  if (k == 0) return CLIFF_OK;
  if (!qubits) return fail(CLIFF_EINVAL, "cliff_measure_async: NULL qubits");
  if (k > t->d.n) return fail(CLIFF_EINVAL, "cliff_measure_async: k = %zu > n = %u", k, t->d.n);
  DeviceGuard g(t->ctx->device);
  return measure_impl(t, qubits, k, seed, circuit, shot0, m0, nullptr, nullptr, k, 0);
}

extern "C" int cliff_tab_read_outcomes(cliff_tab *t, size_t k, uint8_t *host_out,
                                       uint8_t *host_random) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_tab_read_outcomes: NULL tableau");
  if (k > t->d.n) return fail(CLIFF_EINVAL, "cliff_tab_read_outcomes: k = %zu > n = %u", k, t->d.n);
  if (k == 0) return CLIFF_OK;
  DeviceGuard g(t->ctx->device);
  const uint32_t S = t->d.S;
  hipStream_t st = t->ctx->stream;
  std::vector<uint8_t> out_stage(k * S), kind_stage(k);
  HIP_TRY(hipMemcpyAsync(out_stage.data(), t->dev.out, k * S, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(kind_stage.data(), t->dev.kind, k, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  int arc = check_abort(t);
  if (arc) return arc;
  if (host_out)
    for (size_t i = 0; i < k; ++i)
      for (uint32_t s = 0; s < S; ++s) host_out[size_t(s) * k + i] = out_stage[i * S + s];
  if (host_random) memcpy(host_random, kind_stage.data(), k);
  return CLIFF_OK;
}

extern "C" int cliff_sample(cliff_tab *t, cliff_tab *work, const uint32_t *qubits, size_t k,
                            uint64_t seed, uint64_t circuit, uint64_t shot0, uint8_t *host_out,
                            uint8_t *host_random) {
  if (!t || !work) return fail(CLIFF_EINVAL, "cliff_sample: NULL tableau");
  if (work->d.n != t->d.n) return fail(CLIFF_EINVAL, "cliff_sample: work has n=%u, tab n=%u", work->d.n, t->d.n);
  if (work->ctx->device != t->ctx->device) return fail(CLIFF_EINVAL, "cliff_sample: different devices");
  if (work->base == t->base) return fail(CLIFF_EINVAL, "cliff_sample: work aliases tab");
  if (k && !qubits) return fail(CLIFF_EINVAL, "cliff_sample: NULL qubits");
  DeviceGuard g(t->ctx->device);
  const bool two = work->ctx->stream != t->ctx->stream;
  if (two) HIP_TRY(hipStreamSynchronize(t->ctx->stream));
  HIP_TRY(launch_copy_tab(work->dev, t->dev, work->ctx->stream));
  if (two) {
    // later work on tab's stream (gates, say) must not overtake the copy
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, work->ctx->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(t->ctx->stream, ev, 0);
    const hipError_t e2 = hipEventDestroy(ev);
    HIP_TRY(e);
    HIP_TRY(e2);
  }
  if (k == 0) return CLIFF_OK;
  return measure_impl(work, qubits, k, seed, circuit, shot0, 0, host_out, host_random, k, 0);
}

// ------------------------------------------------------------ export/import ---

extern "C" int cliff_tab_export(cliff_tab *t, uint8_t *x, uint8_t *z, uint8_t *r) {
  if (!t || !x || !z || !r) return fail(CLIFF_EINVAL, "cliff_tab_export: NULL argument");
  const Dims &d = t->d;
  DeviceGuard g(t->ctx->device);
  std::vector<uint64_t> X(size_t(d.n) * d.Wp), Z(size_t(d.n) * d.Wp), R(size_t(d.Wp) * d.S), P(d.Wp);
  hipStream_t st = t->ctx->stream;
  HIP_TRY(hipMemcpyAsync(X.data(), t->dev.X, X.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(Z.data(), t->dev.Z, Z.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(R.data(), t->dev.R, R.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(P.data(), t->dev.P, P.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const uint32_t n = d.n, rows = 2 * n;
  for (uint32_t j = 0; j < n; ++j) {
    const uint64_t *cx = &X[size_t(j) * d.Wp], *cz = &Z[size_t(j) * d.Wp];
    for (uint32_t i = 0; i < rows; ++i) {
      x[size_t(i) * n + j] = uint8_t((cx[i >> 6] >> (i & 63)) & 1u);
      z[size_t(i) * n + j] = uint8_t((cz[i >> 6] >> (i & 63)) & 1u);
    }
  }
  for (uint32_t s = 0; s < d.S; ++s)
    for (uint32_t i = 0; i < rows; ++i)
      r[size_t(s) * rows + i] = uint8_t(((R[size_t(i >> 6) * d.S + s] ^ P[i >> 6]) >> (i & 63)) & 1u);
  return CLIFF_OK;
}

namespace cliff {
// defined beside the other whole-tableau kernels in gates.hip
hipError_t launch_gather_words(const TabDev &t, const uint32_t *words, uint32_t nw, uint64_t *ox, uint64_t *oz,
                               hipStream_t st);
}  // namespace cliff

extern "C" int cliff_tab_export_rows(cliff_tab *t, const uint32_t *rows, size_t k, uint8_t *x, uint8_t *z,
                                     uint8_t *r) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_tab_export_rows: NULL tableau");
  if (k == 0) return CLIFF_OK;
  if (!rows || !x || !z) return fail(CLIFF_EINVAL, "cliff_tab_export_rows: NULL argument");
  const Dims &d = t->d;
  const uint32_t n = d.n, S = d.S;
  // the 64-row words holding the requested rows, each fetched once
  std::vector<uint32_t> words, slot(k);
  std::unordered_map<uint32_t, uint32_t> index;
  for (size_t i = 0; i < k; ++i) {
    if (rows[i] >= 2 * n) return fail(CLIFF_EINVAL, "cliff_tab_export_rows: row %u >= 2n = %u", rows[i], 2 * n);
    const uint32_t w = rows[i] >> 6;
    auto it = index.find(w);
    if (it == index.end()) it = index.emplace(w, uint32_t(words.size())).first, words.push_back(w);
    slot[i] = it->second;
  }
  DeviceGuard g(t->ctx->device);
  hipStream_t st = t->ctx->stream;
  const size_t nw = words.size();
  std::vector<uint64_t> cx(nw * n), cz(nw * n), Rw(r ? nw * S : 0), Pw(r ? nw : 0);
  // word w of every column (n words, a column stride of Wp words apart),
  // gathered on the device into [word][column] and copied back in one piece
  const size_t wbytes = align256(nw * 4), cbytes = nw * n * 8;
  char *buf = nullptr;
  HIP_TRY(hipMalloc(&buf, wbytes + 2 * cbytes));
  uint32_t *dw = reinterpret_cast<uint32_t *>(buf);
  uint64_t *dx = reinterpret_cast<uint64_t *>(buf + wbytes), *dz = dx + nw * n;
  hipError_t e = hipMemcpyAsync(dw, words.data(), nw * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_gather_words(t->dev, dw, uint32_t(nw), dx, dz, st);
  if (e == hipSuccess) e = hipMemcpyAsync(cx.data(), dx, cbytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(cz.data(), dz, cbytes, hipMemcpyDeviceToHost, st);
  for (size_t q = 0; r && q < nw && e == hipSuccess; ++q) {
    const uint32_t w = words[q];
    e = hipMemcpyAsync(Rw.data() + q * S, t->dev.R + size_t(w) * S, size_t(S) * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(Pw.data() + q, t->dev.P + w, 8, hipMemcpyDeviceToHost, st);
  }
  const hipError_t es = hipStreamSynchronize(st);
  (void)hipFree(buf);
  HIP_TRY(e);
  HIP_TRY(es);
  for (size_t i = 0; i < k; ++i) {
    const uint32_t sh = rows[i] & 63;
    const uint64_t *px = cx.data() + size_t(slot[i]) * n, *pz = cz.data() + size_t(slot[i]) * n;
    for (uint32_t j = 0; j < n; ++j) {
      x[i * n + j] = uint8_t((px[j] >> sh) & 1u);
      z[i * n + j] = uint8_t((pz[j] >> sh) & 1u);
    }
    if (r)
      for (uint32_t s = 0; s < S; ++s)
        r[size_t(s) * k + i] = uint8_t(((Rw[size_t(slot[i]) * S + s] ^ Pw[slot[i]]) >> sh) & 1u);
  }
  return CLIFF_OK;
}

extern "C" int cliff_tab_import(cliff_tab *t, const uint8_t *x, const uint8_t *z, const uint8_t *r) {
  if (!t || !x || !z || !r) return fail(CLIFF_EINVAL, "cliff_tab_import: NULL argument");
  const Dims &d = t->d;
  const uint32_t n = d.n, rows = 2 * n;
  std::vector<uint64_t> X(size_t(n) * d.Wp, 0), Z(size_t(n) * d.Wp, 0), R(size_t(d.Wp) * d.S, 0),
      P(d.Wp, 0);
  for (uint32_t i = 0; i < rows; ++i)
    for (uint32_t j = 0; j < n; ++j) {
      if (x[size_t(i) * n + j] & 1u) X[size_t(j) * d.Wp + (i >> 6)] |= 1ull << (i & 63);
      if (z[size_t(i) * n + j] & 1u) Z[size_t(j) * d.Wp + (i >> 6)] |= 1ull << (i & 63);
    }
  for (uint32_t s = 0; s < d.S; ++s)
    for (uint32_t i = 0; i < rows; ++i)
      if (r[size_t(s) * rows + i] & 1u) R[size_t(i >> 6) * d.S + s] |= 1ull << (i & 63);
  DeviceGuard g(t->ctx->device);
  hipStream_t st = t->ctx->stream;
  HIP_TRY(hipMemcpyAsync(t->dev.X, X.data(), X.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(t->dev.Z, Z.data(), Z.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(t->dev.R, R.data(), R.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(t->dev.P, P.data(), P.size() * 8, hipMemcpyHostToDevice, st));
  const uint32_t zero = 0;
  HIP_TRY(hipMemcpyAsync(t->dev.abort_flag, &zero, 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CLIFF_OK;
}

extern "C" int cliff_tab_anomalies(cliff_tab *t, uint64_t *count) {
  if (!t || !count) return fail(CLIFF_EINVAL, "cliff_tab_anomalies: NULL argument");
  DeviceGuard g(t->ctx->device);
  int arc = check_abort(t);
  if (arc) return arc;
  uint32_t v = 0;
  HIP_TRY(hipMemcpyAsync(&v, t->dev.state + ST_ANOMALY, 4, hipMemcpyDeviceToHost, t->ctx->stream));
  HIP_TRY(hipStreamSynchronize(t->ctx->stream));
  *count = v;
  return CLIFF_OK;
}

// ------------------------------------------------------- profiling/counters ---

extern "C" int cliff_ctx_profile(cliff_ctx *c, int enable) {
  if (!c) return fail(CLIFF_EINVAL, "cliff_ctx_profile: NULL context");
  DeviceGuard g(c->device);
  HIP_TRY(c->prof.resolve());
  c->prof.reset();
  c->prof.on = enable != 0;
  return CLIFF_OK;
}

extern "C" int cliff_ctx_profile_read(cliff_ctx *c, int kind, double *ms, uint64_t *launches) {
  if (!c || !ms || !launches) return fail(CLIFF_EINVAL, "cliff_ctx_profile_read: NULL argument");
  if (kind < 0 || kind >= kProfKinds) return fail(CLIFF_EINVAL, "cliff_ctx_profile_read: kind %d", kind);
  DeviceGuard g(c->device);
  HIP_TRY(c->prof.resolve());
  *ms = c->prof.ms[kind];
  *launches = c->prof.launches[kind];
  return CLIFF_OK;
}

extern "C" int cliff_tab_counters(cliff_tab *t, uint64_t *out4) {
  if (!t || !out4) return fail(CLIFF_EINVAL, "cliff_tab_counters: NULL argument");
  DeviceGuard g(t->ctx->device);
  int arc = check_abort(t);
  if (arc) return arc;
  uint32_t st[kStateWords];
  HIP_TRY(hipMemcpyAsync(st, t->dev.state, sizeof st, hipMemcpyDeviceToHost, t->ctx->stream));
  HIP_TRY(hipStreamSynchronize(t->ctx->stream));
  uint64_t support;
  memcpy(&support, st + ST_SUPPORT, 8);
  const uint64_t n = t->d.n, W = t->d.W, nr = st[ST_RANDOM_CNT], nd = st[ST_DET_CNT];
  out4[0] = st[ST_ANOMALY];
  out4[1] = nr;
  out4[2] = nd;
  out4[3] = 8 * W * (support + 3 * nr) + 80 * n * nr + 8 * n * W * nd;
  return CLIFF_OK;
}

extern "C" int cliff_tab_reset_counters(cliff_tab *t) {
  if (!t) return fail(CLIFF_EINVAL, "cliff_tab_reset_counters: NULL tableau");
  DeviceGuard g(t->ctx->device);
  HIP_TRY(launch_clear_state(t->dev, t->ctx->stream));
  return CLIFF_OK;
}

// ------------------------------------------------------------------ batch ---

static_assert(sizeof(cliff_batch_desc) == 48, "descriptor layout");

extern "C" size_t cliff_batch_work_bytes(void) { return 256; }

extern "C" int cliff_batch_run(cliff_ctx *c, const cliff_batch_desc *dev_descs,
                               const uint64_t *dev_ops, const uint32_t *dev_offs, uint8_t *dev_out,
                               const uint32_t *dev_order, uint32_t count, uint64_t seed,
                               void *dev_work, uint32_t team, uint32_t maxn, uint32_t max_shots) {
  if (!c || !dev_work || (count && (!dev_descs || !dev_ops || !dev_offs || !dev_out || !dev_order)))
    return fail(CLIFF_EINVAL, "cliff_batch_run: NULL argument");
  if (count == 0) return CLIFF_OK;
  DeviceGuard g(c->device);
  c->prof.begin(PK_BATCH, c->stream);
  hipError_t e = launch_batch(dev_descs, dev_ops, dev_offs, dev_out, dev_order, count, seed,
                              reinterpret_cast<uint32_t *>(dev_work), team, maxn, max_shots, c->num_cus,
                              c->stream);
  c->prof.end(PK_BATCH, c->stream);
  if (e == hipErrorInvalidValue)
    return fail(CLIFF_EINVAL, "cliff_batch_run: team=%u maxn=%u max_shots=%u out of range", team, maxn,
                max_shots);
  HIP_TRY(e);
  return CLIFF_OK;
}

extern "C" int cliff_batch_order_ops(uint32_t n, uint64_t *ops, const uint32_t *offs, uint32_t depth) {
  if (batch_order_ops(n, ops, offs, depth) != 0)
    return fail(CLIFF_EINVAL, "cliff_batch_order_ops: n=%u outside 1..256, or NULL or decreasing offsets", n);
  return CLIFF_OK;
}

extern "C" int cliff_batch_status(cliff_ctx *c, const void *dev_work, uint64_t *out2) {
  if (!c || !dev_work || !out2) return fail(CLIFF_EINVAL, "cliff_batch_status: NULL argument");
  DeviceGuard g(c->device);
  uint32_t v[4];
  HIP_TRY(hipMemcpyAsync(v, dev_work, sizeof v, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  out2[0] = v[1];
  out2[1] = v[2];
  return CLIFF_OK;
}

// ------------------------------------------------------------------ graphs ---

struct cliff_graph {
  int device = 0;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" int cliff_graph_begin(cliff_ctx *c) {
  if (!c) return fail(CLIFF_EINVAL, "cliff_graph_begin: NULL context");
  if (!c->stream) return fail(CLIFF_EINVAL, "cliff_graph_begin: the default stream cannot be captured");
  DeviceGuard g(c->device);
  HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  return CLIFF_OK;
}

extern "C" int cliff_graph_end(cliff_ctx *c, cliff_graph **out) {
  if (!c || !out) return fail(CLIFF_EINVAL, "cliff_graph_end: NULL argument");
  *out = nullptr;
  DeviceGuard g(c->device);
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamEndCapture(c->stream, &graph));
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(CLIFF_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  cliff_graph *gr = new (std::nothrow) cliff_graph();
  if (!gr) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return fail(CLIFF_ENOMEM, "cliff_graph_end: host allocation failed");
  }
  gr->device = c->device;
  gr->stream = c->stream;
  gr->graph = graph;
  gr->exec = exec;
  *out = gr;
  return CLIFF_OK;
}

extern "C" int cliff_graph_launch(cliff_graph *gr) {
  if (!gr) return fail(CLIFF_EINVAL, "cliff_graph_launch: NULL graph");
  DeviceGuard g(gr->device);
  HIP_TRY(hipGraphLaunch(gr->exec, gr->stream));
  return CLIFF_OK;
}

extern "C" int cliff_graph_destroy(cliff_graph *gr) {
  if (!gr) return CLIFF_OK;
  DeviceGuard g(gr->device);
  (void)hipStreamSynchronize(gr->stream);
  if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
  if (gr->graph) (void)hipGraphDestroy(gr->graph);
  delete gr;
  return CLIFF_OK;
}
