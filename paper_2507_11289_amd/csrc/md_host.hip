// md_host.hip -- host runtime and C ABI of libmd (see include/md.h).
//
// Holds the geometry rules (Sec. 4: cells of edge > rc, x-slices of whole cell
// layers), device memory of each simulation, the persistent-launch driver with its
// claim-order tables (Sec. 3.3 / Table 1 generalised to one GPU), the synchronous
// read-back pass, and the serving engine that packs independent runs into shared
// persistent launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../include/md.h"
#include "md_internal.h"

using namespace mdk;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(MD_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

extern "C" const char* md_strerror(int status) {
  switch (status) {
    case MD_OK: return "ok";
    case MD_PENDING: return "pending";
    case MD_EINVAL: return "invalid argument";
    case MD_ENOMEM: return "out of memory";
    case MD_EHIP: return "HIP runtime error";
    case MD_ESTATE: return "call out of order or poisoned handle";
    case MD_ECAPACITY: return "cell capacity exceeded";
    case MD_EUNSTABLE: return "unstable trajectory (non-finite value or slice jump)";
    case MD_ENOTFOUND: return "unknown ticket";
    case MD_EBUSY: return "busy";
    case MD_EWATCHDOG: return "device wait exceeded its time budget";
    default: return "unknown status";
  }
}

extern "C" const char* md_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// geometry (Sec. 4: N_xyz = floor(b / rc) cells per edge, edge l = b / N_xyz > rc;
// slices perpendicular to x, each holding whole cell layers)
// ---------------------------------------------------------------------------
static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

static int make_geom(const double box[3], int slices, double rc, double dt, int prec, DGeom* g) {
  if (!box) return fail(MD_EINVAL, "box is NULL");
  if (!finite_pos(rc)) return fail(MD_EINVAL, "rc must be finite and > 0");
  if (!finite_pos(dt)) return fail(MD_EINVAL, "dt must be finite and > 0");
  if (prec != MD_FP64 && prec != MD_FP32_FORCE) return fail(MD_EINVAL, "unknown precision %d", prec);
  if (slices < 3) return fail(MD_EINVAL, "need at least 3 slices (got %d)", slices);
  for (int d = 0; d < 3; d++)
    if (!finite_pos(box[d])) return fail(MD_EINVAL, "box[%d] must be finite and > 0", d);
  if (box[0] / slices < rc) return fail(MD_EINVAL, "slice width Lx/S = %g is below rc", box[0] / slices);
  const double margin = 1.0 + std::ldexp(1.0, -40);
  long long ncx = (long long)std::floor((box[0] / slices) / rc);
  if (box[0] / (double)(slices * ncx) < rc * margin) ncx -= 1;
  long long gy = (long long)std::floor(box[1] / rc);
  if (gy > 0 && box[1] / (double)gy < rc * margin) gy -= 1;
  long long gz = (long long)std::floor(box[2] / rc);
  if (gz > 0 && box[2] / (double)gz < rc * margin) gz -= 1;
  if (ncx < 1) return fail(MD_EINVAL, "slice width too close to rc");
  if (gy < 3 || gz < 3) return fail(MD_EINVAL, "fewer than 3 cells along y or z");
  const long long cps = ncx * gy * gz;
  const long long ncell = cps * slices;
  if (ncell > (1ll << 26) || slices > 32767)
    return fail(MD_EINVAL, "grid too large (%lld cells, %d slices)", ncell, slices);
  std::memset(g, 0, sizeof(*g));
  g->S = slices;
  g->ncx = (int)ncx;
  g->G[0] = (int)(slices * ncx);
  g->G[1] = (int)gy;
  g->G[2] = (int)gz;
  for (int d = 0; d < 3; d++) {
    g->L[d] = box[d];
    g->halfL[d] = 0.5 * box[d];
    g->l[d] = box[d] / (double)g->G[d];
    g->inv_l[d] = 1.0 / g->l[d];
    g->inv_G[d] = 1.0 / (double)g->G[d];
  }
  g->inv_ncx = 1.0 / (double)g->ncx;
  g->inv_cps = 1.0 / (double)cps;
  g->rc2 = rc * rc;
  const double ir2 = 1.0 / g->rc2;
  const double ir6 = ir2 * ir2 * ir2;
  g->uc = 4.0 * ir6 * (ir6 - 1.0);
  g->dt = dt;
  g->hdt = 0.5 * dt;
  // FP32 guard band: |r2_fp32 - rc^2| <= 2^-16 rc^2 is decided again in FP64.
  const double lo = g->rc2 * (1.0 - std::ldexp(1.0, -16));
  const double hi = g->rc2 * (1.0 + std::ldexp(1.0, -16));
  float flo = (float)lo, fhi = (float)hi;
  if ((double)flo > lo) flo = std::nextafter(flo, 0.0f);
  if ((double)fhi < hi) fhi = std::nextafter(fhi, 1e30f);
  g->rc2_lo_f = flo;
  g->rc2_hi_f = fhi;
  // Pre-filter threshold.  The FP32 force pass estimates r2 - pre on the matrix cores
  // as |q_c|^2 - 2 q_a.q_c + (|q_a|^2 - pre), from staged coordinates q relative to the
  // block origin (|x| <= 2 lx, |y| <= 2 ly, |z| <= (BLOCK_CELLS + 1) lz, so |q|^2 <= M).
  // Whatever the order and rounding of its sums, that estimate is within
  // 2^-24 (31 M + 7 pre) of the exact r2 - pre; the threshold lies 2^-10 rc^2 above the
  // guard band plus 2^-18 (M + hi), more than twice that, so every pair the exact FP32
  // arithmetic puts at or below the band is marked.
  const double M = 1.01 * (4.0 * g->l[0] * g->l[0] + 4.0 * g->l[1] * g->l[1] +
                           (double)((BLOCK_CELLS + 1) * (BLOCK_CELLS + 1)) * g->l[2] * g->l[2]);
  g->rc2_pre_f = (float)(hi * (1.0 + std::ldexp(1.0, -10)) + std::ldexp(M + hi, -18));
  g->rc2_f = (float)g->rc2;
  g->uc_f = (float)g->uc;
  g->cps = (int)cps;
  g->ncell = (int)ncell;
  g->prec = prec;
  g->cap = CELL_CAP;
  return MD_OK;
}

// Finalise items per slice and step are the force items' count divided by this (rounded
// up) under the dataflow scheduler.
constexpr int64_t FINALISE_MERGE = 4;
// Served runs: cells per work item (short items keep each step's critical path short)
// and steps per packed launch when the server is given no quantum.
constexpr int64_t SERVED_CHUNK_MIN = 32, SERVED_CHUNK_MAX = 64;
// Cells per work item of a served run: a quarter of a slice, within [32, 64] cells: small
// runs keep four items per slice (a short critical path per step), large runs take items
// of 64 cells (fewer, so less per-item overhead).
static int64_t served_chunk_cells(const DGeom& g) {
  return std::min<int64_t>(SERVED_CHUNK_MAX, std::max<int64_t>(SERVED_CHUNK_MIN, g.cps / 4));
}
constexpr int64_t SERVED_QUANTUM = 64;

static int64_t finalise_items(int64_t nch) {
  return std::max<int64_t>(1, (nch + FINALISE_MERGE - 1) / FINALISE_MERGE);
}

// Device bytes of one simulation with `nch` force items per slice, advanced in launches of
// at most `launch_steps` steps: the resident state plus the largest transient buffers.
//   resident: two cell buffers, the cell counters of both parities, per-slice counters,
//     cumulative migrations, claim table;
//   transient, never at the same time: the load copies (pos, vel) or the read-back outputs
//     (pos, vel, force), at most 72 B per atom, plus the read-back energy partials;
//   per launch: the work queue (8 B per item), the energy partials of one sample, the
//     migration log of every step of the launch;
//   thermostat: the forces kept between force and integrate items (24 B per slot) and the
//     per-item kinetic energies.
static int64_t footprint(const DGeom& g, int64_t n, int64_t nch, int64_t launch_steps, bool thermo) {
  int64_t b = 2ll * g.ncell * CELL_BYTES;
  b += 4ll * g.ncell * 4;
  b += 64ll * g.S + 4096;
  b += 3ll * 3 * 8 * n + 3ll * 8 * sync_blocks(g);
  const int64_t ips = g.S * (nch + finalise_items(nch) + (thermo ? nch : 0));
  b += launch_steps * ips * 8;
  b += 3ll * 8 * g.S * nch;
  b += 2ll * 4 * g.S * launch_steps;
  if (thermo) b += (int64_t)g.ncell * 3 * CELL_CAP * 8 + 16ll * g.S * nch;
  return b;
}

static int auto_chunks(const DGeom& g, int64_t chunk_cells, int64_t n_atoms);

// Footprint of a served run: served_chunk_cells per item, `quantum` steps per launch.
static int64_t served_footprint(const DGeom& g, int64_t n, int64_t quantum) {
  return footprint(g, n, auto_chunks(g, served_chunk_cells(g), n), quantum > 0 ? quantum : SERVED_QUANTUM, false);
}

extern "C" int64_t md_footprint_bytes(const double box[3], int slices, double rc, int64_t n) {
  DGeom g;
  if (make_geom(box, slices, rc, 1.0, MD_FP64, &g) != MD_OK) return -1;
  return served_footprint(g, n, 0);
}

// ---------------------------------------------------------------------------
// claim orders (one step = 2S entries: (phase << 15) | slice; phase 0 = force /
// integrate of step k, phase 1 = finalise of step k+1).  A finalise entry of slice i
// must follow the integrate entries of i-1, i, i+1.
// ---------------------------------------------------------------------------
static std::vector<uint16_t> make_order(int S, int kind, uint64_t seed) {
  std::vector<uint16_t> o;
  o.reserve(2 * S);
  auto P2 = [](int s) { return (uint16_t)s; };
  auto P1 = [](int s) { return (uint16_t)((1u << 15) | (unsigned)s); };
  if (kind == MD_ORDER_PHASED) {
    for (int s = 0; s < S; s++) o.push_back(P2(s));
    for (int s = 0; s < S; s++) o.push_back(P1(s));
  } else if (kind == MD_ORDER_SWEEP || kind == MD_ORDER_DESCENDING) {
    std::vector<int> seq(S);
    for (int i = 0; i < S; i++) seq[i] = kind == MD_ORDER_SWEEP ? i : S - 1 - i;
    // integrate slices in sweep order; finalise slice seq[i-1] right after seq[i] is
    // integrated (its other neighbour seq[i-2] is already done); the first slice waits
    // for the last one (periodic)
    o.push_back(P2(seq[0]));
    o.push_back(P2(seq[1]));
    for (int i = 2; i < S; i++) {
      o.push_back(P2(seq[i]));
      o.push_back(P1(seq[i - 1]));
    }
    o.push_back(P1(seq[S - 1]));
    o.push_back(P1(seq[0]));
  } else {
    std::mt19937_64 rng(seed);
    std::vector<int> done(S, 0), fin(S, 0);
    std::vector<uint16_t> ready;
    for (int s = 0; s < S; s++) ready.push_back(P2(s));
    while (!ready.empty()) {
      size_t pick = (size_t)(rng() % ready.size());
      uint16_t e = ready[pick];
      ready.erase(ready.begin() + (long)pick);
      o.push_back(e);
      if ((e >> 15) == 0) {
        int s = e & 0x7fff;
        done[s] = 1;
        for (int q = -1; q <= 1; q++) {
          int t = (s + q + S) % S;
          if (!fin[t] && done[(t + S - 1) % S] && done[t] && done[(t + 1) % S]) {
            fin[t] = 1;
            ready.push_back(P1(t));
          }
        }
      }
    }
  }
  return o;
}

extern "C" int md_claim_table(int slices, int order, uint64_t seed, uint16_t* out) {
  if (slices < 3 || slices > 32767 || !out) return fail(MD_EINVAL, "bad arguments");
  if (order < MD_ORDER_SWEEP || order > MD_ORDER_RANDOM) return fail(MD_EINVAL, "no table for this order");
  std::vector<uint16_t> t = make_order(slices, order, seed);
  std::memcpy(out, t.data(), t.size() * sizeof(uint16_t));
  return MD_OK;
}

// Multi-time-level sweep (MD_ORDER_WAVEFRONT): the entries of `levels` consecutive steps,
// (j << 16) | (phase << 15) | slice, sorted by key.  Integrate of slice i at step j has key
// 6j + 2d(i), finalise of slice i for step j+1 has key 6j + 2 max(d(i-1), d(i), d(i+1)) + 1,
// d(i) = min(i, S - i).  Finalise keys exceed the keys of the integrates they need, and
// integrate of step j+1 (key 6j + 6 + 2d(i)) exceeds every finalise it needs (at most
// 6j + 2(d(i) + 2) + 1, since d changes by at most one between neighbours).
constexpr int MAX_WAVEFRONT_LEVELS = 64;
static std::vector<uint32_t> make_wavefront(int S, int levels) {
  struct E {
    long key;
    uint32_t v;
  };
  std::vector<E> e;
  e.reserve((size_t)2 * S * levels);
  auto d = [S](int i) { i = ((i % S) + S) % S; return std::min(i, S - i); };
  for (int j = 0; j < levels; j++)
    for (int i = 0; i < S; i++) {
      e.push_back({6l * j + 2l * d(i), ((uint32_t)j << 16) | (uint32_t)i});
      const int m = std::max(d(i - 1), std::max(d(i), d(i + 1)));
      e.push_back({6l * j + 2l * m + 1, ((uint32_t)j << 16) | (1u << 15) | (uint32_t)i});
    }
  std::stable_sort(e.begin(), e.end(), [](const E& a, const E& b) {
    if (a.key != b.key) return a.key < b.key;
    return (a.v & 0xffffu) < (b.v & 0xffffu);
  });
  std::vector<uint32_t> out(e.size());
  for (size_t k = 0; k < e.size(); k++) out[k] = e[k].v;
  return out;
}

extern "C" int md_wavefront_table(int slices, int levels, uint32_t* out) {
  if (slices < 3 || slices > 32767 || levels < 1 || levels > MAX_WAVEFRONT_LEVELS || !out)
    return fail(MD_EINVAL, "bad arguments");
  std::vector<uint32_t> t = make_wavefront(slices, levels);
  std::memcpy(out, t.data(), t.size() * sizeof(uint32_t));
  return MD_OK;
}

// ---------------------------------------------------------------------------
// device buffers of one simulation / run
// ---------------------------------------------------------------------------
// Device memory comes from hipMalloc, or from the caller's allocator (md_set_allocator),
// which may only change while no simulation or server exists.
static md_alloc_fn g_alloc = nullptr;
static md_free_fn g_free = nullptr;
static void* g_alloc_ctx = nullptr;
static std::atomic<int> g_live{0};  // simulations and servers alive
static std::mutex g_alloc_mu;

// Counts a handle as alive from its creation on; a failed creation gives the count back.
struct LiveGuard {
  bool keep = false;
  LiveGuard() { g_live++; }
  ~LiveGuard() {
    if (!keep) g_live--;
  }
};

extern "C" int md_set_allocator(md_alloc_fn alloc, md_free_fn release, void* ctx) {
  if ((alloc == nullptr) != (release == nullptr))
    return fail(MD_EINVAL, "give both an allocation and a release function, or neither");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if (g_live.load() != 0)
    return fail(MD_ESTATE, "%d simulations or servers still hold device memory", g_live.load());
  g_alloc = alloc;
  g_free = release;
  g_alloc_ctx = alloc ? ctx : nullptr;
  return MD_OK;
}

template <class T>
static int dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  const size_t bytes = count * sizeof(T);
  if (g_alloc) {
    void* q = g_alloc(bytes, g_alloc_ctx);
    if (!q) return fail(MD_ENOMEM, "the caller's allocator returned no memory for %zu bytes", bytes);
    if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {
      g_free(q, g_alloc_ctx);
      return fail(MD_EINVAL, "the caller's allocator returned memory not aligned to 256 bytes");
    }
    *p = static_cast<T*>(q);
    return MD_OK;
  }
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(MD_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  }
  return MD_OK;
}

template <class T>
static void dfree(T*& p) {
  if (p) {
    if (g_free) g_free((void*)p, g_alloc_ctx);
    else (void)hipFree((void*)p);
  }
  p = nullptr;
}

// ---------------------------------------------------------------------------
// Launch scratch that is never allocated (md_step_noalloc): the run arguments, work
// queue, energy partials and migration log of its launches are carved out of one fixed
// array per GPU, which the process holds until it ends.  In host code `scratch` names a
// host-side stand-in, not device memory: everything that reaches a kernel or a copy uses
// the device address looked up once per device by scratch_setup.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[MD_NOALLOC_SCRATCH_BYTES];
constexpr int SCRATCH_MAX_DEVICES = 64;
static unsigned char* g_scratch_dev[SCRATCH_MAX_DEVICES];  // device address of `scratch` per GPU
static std::mutex g_scratch_mu;

// With device `dev` current: look up this GPU's copy of the array (once per device).
static int scratch_setup(int dev) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    return fail(MD_EHIP, "device %d is beyond the %d devices the launch scratch supports", dev,
                SCRATCH_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return MD_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    return fail(MD_EHIP, "hipGetSymbolAddress of the launch scratch failed: %s", hipGetErrorString(e));
  }
  g_scratch_dev[dev] = static_cast<unsigned char*>(ptr);
  return MD_OK;
}

static size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

// Consecutive 256-byte aligned pieces of a fixed device region.
struct Carve {
  unsigned char* base;
  size_t cap;
  size_t used;
  template <class T> T* take(size_t count) {
    const size_t need = round256(std::max<size_t>(count, 1) * sizeof(T));
    if (need > cap - used) return nullptr;
    T* p = reinterpret_cast<T*>(base + used);
    used += need;
    return p;
  }
};

struct SimBuffers {
  unsigned char* cells[2] = {nullptr, nullptr};
  uint32_t* ncnt[2] = {nullptr, nullptr};
  uint32_t* nin[2] = {nullptr, nullptr};
  uint32_t* cntA = nullptr;
  uint32_t* cntF = nullptr;
  uint32_t* cntK = nullptr;
  uint32_t* err = nullptr;
  uint32_t* abort = nullptr;
  unsigned long long* migcum = nullptr;
  unsigned long long* paircnt = nullptr;
  unsigned long long* scount = nullptr;  // atoms per slice (work-queue ranges, md_get_slice_counts)
  uint32_t* order = nullptr;  // claim table of one round (up to MAX_WAVEFRONT_LEVELS steps)
  int order_len = 0;

  int alloc(const DGeom& g) {
    int rc;
    for (int p = 0; p < 2; p++) {
      if ((rc = dalloc(&cells[p], (size_t)g.ncell * CELL_BYTES))) return rc;
      if ((rc = dalloc(&ncnt[p], (size_t)g.ncell))) return rc;
      if ((rc = dalloc(&nin[p], (size_t)g.ncell))) return rc;
    }
    if ((rc = dalloc(&cntA, (size_t)g.S))) return rc;
    if ((rc = dalloc(&cntF, (size_t)g.S))) return rc;
    if ((rc = dalloc(&cntK, (size_t)g.S))) return rc;
    if ((rc = dalloc(&err, 1))) return rc;
    if ((rc = dalloc(&abort, 1))) return rc;
    if ((rc = dalloc(&migcum, (size_t)2 * g.S))) return rc;
    if ((rc = dalloc(&paircnt, 2))) return rc;
    if ((rc = dalloc(&scount, (size_t)g.S))) return rc;
    if ((rc = dalloc(&order, (size_t)2 * g.S * MAX_WAVEFRONT_LEVELS))) return rc;
    order_len = 2 * g.S * MAX_WAVEFRONT_LEVELS;
    return MD_OK;
  }
  void release() {
    for (int p = 0; p < 2; p++) {
      dfree(cells[p]);
      dfree(ncnt[p]);
      dfree(nin[p]);
    }
    dfree(cntA);
    dfree(cntF);
    dfree(cntK);
    dfree(err);
    dfree(abort);
    dfree(migcum);
    dfree(paircnt);
    dfree(scount);
    dfree(order);
  }
};

struct LaunchScratch {
  RunArgs* d_runs = nullptr;
  uint32_t* d_errs = nullptr;  // error word of every run after a launch
  size_t runs_cap = 0;
  long long* d_round_base = nullptr;
  int* d_round_active = nullptr;
  size_t round_cap = 0;
  long long* d_run_prefix = nullptr;
  unsigned long long* d_ticket = nullptr;
  unsigned long long* d_q = nullptr;
  size_t q_cap = 0;
  unsigned long long* d_q_tail = nullptr;
  uint32_t* d_launch_err = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};

  int reserve(size_t nruns, size_t nrounds) {
    int rc;
    if (!d_ticket && (rc = dalloc(&d_ticket, (size_t)MAX_XQ * XQ_STRIDE))) return rc;
    if (!d_q_tail && (rc = dalloc(&d_q_tail, (size_t)MAX_XQ * XQ_STRIDE))) return rc;
    if (!d_launch_err && (rc = dalloc(&d_launch_err, 1))) return rc;
    if (nruns > runs_cap) {
      dfree(d_runs);
      dfree(d_run_prefix);
      dfree(d_errs);
      if ((rc = dalloc(&d_runs, nruns)) || (rc = dalloc(&d_run_prefix, nruns + 1)) || (rc = dalloc(&d_errs, nruns)))
        return rc;
      runs_cap = nruns;
    }
    if (nrounds + 1 > round_cap) {
      dfree(d_round_base);
      dfree(d_round_active);
      if ((rc = dalloc(&d_round_base, nrounds + 1)) || (rc = dalloc(&d_round_active, nrounds + 1))) return rc;
      round_cap = nrounds + 1;
    }
    return MD_OK;
  }
  void release() {
    dfree(d_runs);
    dfree(d_errs);
    dfree(d_round_base);
    dfree(d_round_active);
    dfree(d_run_prefix);
    dfree(d_ticket);
    dfree(d_q);
    dfree(d_q_tail);
    dfree(d_launch_err);
    q_cap = 0;
    for (int i = 0; i < 2; i++)
      if (ev[i]) (void)hipEventDestroy(ev[i]);
    ev[0] = ev[1] = nullptr;
    runs_cap = round_cap = 0;
  }
};

struct md_sim {
  DGeom g{};
  double rc = 0, dt = 0;
  int prec = 0;
  int64_t n = 0;
  int64_t t = 0;
  int par = 0;       // parity of the sorted buffer of step t
  int first = 1;     // stored velocities are v(t) (just loaded)
  bool loaded = false;
  bool poisoned = false;
  SimBuffers b;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  // options
  int64_t every = 0;
  int order_kind = MD_ORDER_DATAFLOW;
  uint64_t order_seed = 1;
  bool order_dirty = true;
  int wlev = 4;               // MD_OPT_WAVEFRONT_LEVELS
  int order_wlev = 0;         // steps per round of the uploaded table
  bool miglog_on = false;
  int64_t chunk_cells = 0;
  bool count_pairs = false;
  int64_t watchdog_ms = 20000;
  int64_t grid_override = 0;
  int64_t fail_at = -1;
  int64_t max_steps_per_launch = 4096;
  double thermo_T = 0.0;  // velocity-scaling thermostat target (0: off)
  bool trace_on = false;
  std::vector<TraceRec> trace;
  TraceRec* d_trace = nullptr;
  size_t trace_cap = 0;
  int nch = 1;
  // last md_step
  std::vector<double> elog;
  std::vector<int32_t> miglog;
  int64_t miglog_steps = 0;
  int64_t cand = 0, inr = 0, counted = 0;
  double last_seconds = 0;
  double last_kernel_seconds = 0;
  int last_launches = 0;
  int last_grid = 0;
  // launch scratch (device)
  LaunchScratch* ls = nullptr;
  double* d_epart = nullptr;
  size_t epart_cap = 0;
  uint32_t* d_miglog = nullptr;
  size_t miglog_cap = 0;
  double* d_fbuf = nullptr;   // thermostat: forces between the force and integrate items
  double* d_kpart = nullptr;  // thermostat: per-item kinetic energy and atom count
  size_t kpart_cap = 0;
  // energy partials and migration log of the current launch (own buffers or scratch)
  double* cur_epart = nullptr;
  uint32_t* cur_miglog = nullptr;
  int dev = 0;  // device current at md_init
  // XCD work queues: XCDs of the device (1: one queue), whether md_step uses them, and the
  // slice ranges of the queues for the current md_step
  int nxcc = 1;
  bool xcd_queues = false;
  int nq = 1;
  int xfirst[MAX_XQ + 1] = {0};
};

static int device_ready() {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count < 1) {
    (void)hipGetLastError();
    return fail(MD_EHIP, "no HIP device available (%s)", hipGetErrorString(e));
  }
  return MD_OK;
}

// Work items per slice and phase.  Without a given cell count an item holds about
// ATOMS_PER_ITEM atoms (at least 32 cells): fewer, larger items mean fewer queue
// operations and fewer L2 invalidations at item start, more and smaller ones balance
// better; these sizes were the fastest on the homogeneous and slab workloads.
static int auto_chunks(const DGeom& g, int64_t chunk_cells, int64_t n_atoms) {
  int64_t nch;
  if (chunk_cells > 0) {
    nch = (g.cps + chunk_cells - 1) / chunk_cells;
  } else {
    const double atoms_per_item = g.prec == 1 ? 2200.0 : 1900.0;
    nch = std::llround((double)n_atoms / ((double)g.S * atoms_per_item));
    nch = std::min<int64_t>(nch, (g.cps + 31) / 32);
  }
  if (nch < 1) nch = 1;
  if (nch > g.cps) nch = g.cps;
  if (nch > 4096) nch = 4096;
  return (int)nch;
}

static void free_launch_scratch(md_sim* s) {
  if (s->ls) {
    s->ls->release();
    delete s->ls;
    s->ls = nullptr;
  }
  dfree(s->d_epart);
  dfree(s->d_miglog);
  dfree(s->d_trace);
  dfree(s->d_fbuf);
  dfree(s->d_kpart);
  s->epart_cap = s->miglog_cap = s->trace_cap = s->kpart_cap = 0;
}

extern "C" void md_free(md_sim* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  s->b.release();
  free_launch_scratch(s);
  if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
  delete s;
  g_live--;
}

extern "C" int md_init(const double box[3], int slices, double rc, double dt, int precision,
                       md_sim** out) {
  if (!out) return fail(MD_EINVAL, "out is NULL");
  *out = nullptr;
  DGeom g;
  int rc_ = make_geom(box, slices, rc, dt, precision, &g);
  if (rc_) return rc_;
  if ((rc_ = device_ready())) return rc_;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if ((rc_ = scratch_setup(dev))) return rc_;
  LiveGuard live;
  std::unique_ptr<md_sim> s(new md_sim());
  s->g = g;
  s->rc = rc;
  s->dt = dt;
  s->prec = precision;
  s->dev = dev;
  {
    int nx = 1;
    if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || nx < 1 || nx > MAX_XQ) {
      (void)hipGetLastError();
      nx = 1;
    }
    s->nxcc = nx;
  }
  HIPCHK(hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking));
  s->stream = s->own_stream;
  if ((rc_ = s->b.alloc(g))) {
    s->b.release();
    (void)hipStreamDestroy(s->own_stream);
    return rc_;
  }
  s->ls = new LaunchScratch();
  s->nch = auto_chunks(g, 0, 0);
  *out = s.release();
  live.keep = true;
  return MD_OK;
}

extern "C" int md_set_stream(md_sim* s, void* hip_stream) {
  if (!s) return fail(MD_EINVAL, "sim is NULL");
  HIPCHK(hipStreamSynchronize(s->stream));
  s->stream = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : s->own_stream;
  return MD_OK;
}

extern "C" int md_set_thermostat(md_sim* s, double temperature) {
  if (!s) return fail(MD_EINVAL, "sim is NULL");
  if (!std::isfinite(temperature) || temperature < 0.0)
    return fail(MD_EINVAL, "thermostat temperature must be finite and >= 0");
  s->thermo_T = temperature;
  return MD_OK;
}

extern "C" int md_set_option(md_sim* s, int key, int64_t value) {
  if (!s) return fail(MD_EINVAL, "sim is NULL");
  switch (key) {
    case MD_OPT_ENERGY_EVERY:
      if (value < 0) return fail(MD_EINVAL, "energy_every must be >= 0");
      s->every = value;
      return MD_OK;
    case MD_OPT_CLAIM_ORDER:
      if (value < MD_ORDER_SWEEP || value > MD_ORDER_WAVEFRONT) return fail(MD_EINVAL, "unknown claim order");
      s->order_kind = (int)value;
      s->order_dirty = true;
      return MD_OK;
    case MD_OPT_ORDER_SEED:
      s->order_seed = (uint64_t)value;
      s->order_dirty = true;
      return MD_OK;
    case MD_OPT_MIGRATION_LOG:
      s->miglog_on = value != 0;
      return MD_OK;
    case MD_OPT_CHUNK_CELLS:
      if (value < 0) return fail(MD_EINVAL, "chunk cells must be >= 0");
      s->chunk_cells = value;
      s->nch = auto_chunks(s->g, value, s->n);
      return MD_OK;
    case MD_OPT_COUNT_PAIRS:
      s->count_pairs = value != 0;
      return MD_OK;
    case MD_OPT_WATCHDOG_MS:
      if (value <= 0) return fail(MD_EINVAL, "watchdog must be > 0 ms");
      s->watchdog_ms = value;
      return MD_OK;
    case MD_OPT_GRID:
      if (value < 0) return fail(MD_EINVAL, "grid must be >= 0");
      s->grid_override = value;
      return MD_OK;
    case MD_OPT_FAIL_AT_STEP:
      s->fail_at = value;
      return MD_OK;
    case MD_OPT_TRACE:
      s->trace_on = value != 0;
      return MD_OK;
    case MD_OPT_CELL_CAPACITY:
      if (value < 1 || value > CELL_CAP) return fail(MD_EINVAL, "cell capacity must be in [1, %d]", CELL_CAP);
      s->g.cap = (int)value;
      return MD_OK;
    case MD_OPT_WAVEFRONT_LEVELS:
      if (value < 1 || value > MAX_WAVEFRONT_LEVELS)
        return fail(MD_EINVAL, "wavefront levels must be in [1, %d]", MAX_WAVEFRONT_LEVELS);
      s->wlev = (int)value;
      s->order_dirty = true;
      return MD_OK;
    case MD_OPT_XCD_QUEUES:
      s->xcd_queues = value != 0;
      return MD_OK;
    case MD_OPT_MAX_STEPS_PER_LAUNCH:
      if (value <= 0) return fail(MD_EINVAL, "max steps per launch must be > 0");
      s->max_steps_per_launch = value;
      return MD_OK;
    default:
      return fail(MD_EINVAL, "unknown option %d", key);
  }
}

static int check_positions(const DGeom& g, int64_t n, const double* pos, const double* vel) {
  for (int64_t i = 0; i < n; i++) {
    for (int d = 0; d < 3; d++) {
      const double x = pos[3 * i + d], v = vel[3 * i + d];
      if (!std::isfinite(x) || !std::isfinite(v))
        return fail(MD_EINVAL, "atom %lld: non-finite position or velocity", (long long)i);
      if (x < 0.0 || x > g.L[d])
        return fail(MD_EINVAL, "atom %lld: coordinate %d = %.17g outside [0, %.17g]", (long long)i, d, x,
                    g.L[d]);
    }
  }
  return MD_OK;
}

static int read_err(md_sim* s, uint32_t* word) {
  HIPCHK(hipMemcpyAsync(word, s->b.err, sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return MD_OK;
}

static int err_status(uint32_t w) {
  if (w & ERR_CAPACITY) return MD_ECAPACITY;
  if (w & ERR_WATCHDOG) return MD_EWATCHDOG;
  if (w & (ERR_NONFINITE | ERR_DISPLACEMENT | ERR_INJECTED)) return MD_EUNSTABLE;
  if (w & ERR_BADINPUT) return MD_EINVAL;
  return MD_OK;
}

static const char* err_text(uint32_t w) {
  if (w & ERR_CAPACITY) return "a cell exceeded its atom slots (MD_OPT_CELL_CAPACITY, at most 64)";
  if (w & ERR_WATCHDOG) return "a dependency wait exceeded the watchdog budget";
  if (w & ERR_DISPLACEMENT) return "an atom moved by more than one slice in one step";
  if (w & ERR_NONFINITE) return "non-finite position, velocity or force";
  if (w & ERR_INJECTED) return "fault injected at the requested step";
  return "device error";
}

// Load an id-ordered state into parity 0: bin on the device, then id order per cell.
static int load_state(md_sim* s, int64_t n, const double* pos, const double* vel, bool device_ptrs) {
  const DGeom& g = s->g;
  hipStream_t st = s->stream;
  for (int p = 0; p < 2; p++) {
    if (launch_clear_u32(s->b.ncnt[p], g.ncell, 0u, st)) return fail(MD_EHIP, "clear failed");
    if (launch_clear_u32(s->b.nin[p], g.ncell, 0u, st)) return fail(MD_EHIP, "clear failed");
  }
  if (launch_clear_u32(s->b.err, 1, 0u, st)) return fail(MD_EHIP, "clear failed");
  if (launch_clear_u32(reinterpret_cast<uint32_t*>(s->b.migcum), 4ll * g.S, 0u, st))
    return fail(MD_EHIP, "clear failed");
  if (n > 0) {
    double *dpos = nullptr, *dvel = nullptr;
    int rc;
    if (device_ptrs) {
      dpos = const_cast<double*>(pos);
      dvel = const_cast<double*>(vel);
    } else {
      if ((rc = dalloc(&dpos, (size_t)3 * n))) return rc;
      if ((rc = dalloc(&dvel, (size_t)3 * n))) {
        dfree(dpos);
        return rc;
      }
      hipError_t e1 = hipMemcpyAsync(dpos, pos, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st);
      hipError_t e2 = hipMemcpyAsync(dvel, vel, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st);
      if (e1 != hipSuccess || e2 != hipSuccess) {
        (void)hipStreamSynchronize(st);
        dfree(dpos);
        dfree(dvel);
        return fail(MD_EHIP, "host-to-device copy failed");
      }
    }
    int l1 = launch_load_scatter(g, dpos, dvel, n, s->b.cells[0], s->b.ncnt[0], s->b.err, st);
    int l2 = launch_sort_cells(g, s->b.cells[0], s->b.ncnt[0], s->b.err, st);
    hipError_t e = hipStreamSynchronize(st);
    if (!device_ptrs) {
      dfree(dpos);
      dfree(dvel);
    }
    if (l1 || l2 || e != hipSuccess) return fail(MD_EHIP, "binning kernels failed: %s", hipGetErrorString(e));
  }
  uint32_t w = 0;
  int rc = read_err(s, &w);
  if (rc) return rc;
  if (w) return fail(err_status(w), "md_load: %s", err_text(w));
  return MD_OK;
}

extern "C" int md_load(md_sim* s, int64_t n, const double* pos, const double* vel) {
  if (!s) return fail(MD_EINVAL, "sim is NULL");
  if (n < 0 || (n > 0 && (!pos || !vel))) return fail(MD_EINVAL, "bad atom arrays");
  if (n >= (int64_t)UINT32_MAX) return fail(MD_EINVAL, "too many atoms");
  int rc = check_positions(s->g, n, pos, vel);
  if (rc) return rc;
  s->loaded = false;
  s->poisoned = false;
  if ((rc = load_state(s, n, pos, vel, false))) {
    s->poisoned = true;
    return rc;
  }
  s->n = n;
  s->nch = auto_chunks(s->g, s->chunk_cells, n);
  s->t = 0;
  s->par = 0;
  s->first = 1;
  s->loaded = true;
  s->elog.clear();
  s->miglog.clear();
  s->miglog_steps = 0;
  return MD_OK;
}

// ---------------------------------------------------------------------------
// packed persistent launch: one or more simulations advance k_r steps each in one
// launch; tickets are dealt round by round (round k holds step k of every run that
// still has steps), so a small run is never starved by a large one.
// ---------------------------------------------------------------------------
static int grid_size(int prec, int kind, int nvt, int64_t override_) {
  if (override_ > 0) return (int)override_;
  int bpc = 1, cus = 1;
  if (persistent_grid(prec, kind, nvt, &bpc, &cus)) return 256;
  return bpc * cus;
}

static long long watchdog_ticks(int64_t ms) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  return (long long)ms * (long long)khz;
}

// Energy samples a launch of k steps from step t takes (steps t' with t' % every == 0).
static void launch_samples(const md_sim* s, int64_t k_steps, int64_t* nsample, int64_t* first_j) {
  *nsample = 0;
  *first_j = 0;
  if (s->every > 0) {
    *first_j = (s->t + s->every - 1) / s->every;
    const int64_t last_j = (s->t + k_steps - 1) / s->every;
    *nsample = last_j >= *first_j ? last_j - *first_j + 1 : 0;
  }
}

// Per-run preparation of a launch of k steps: claim table, energy/migration buffers
// (the run's own, or carved from `arena`), and the device-visible RunArgs.
static int prepare_run(md_sim* s, int64_t k_steps, bool dataflow, hipStream_t st, RunArgs* ra,
                       int64_t* nsample_out, int64_t* first_j_out, Carve* arena, int64_t reserve_steps = 0) {
  const DGeom& g = s->g;
  int rc;
  // claim table of one round: wlev steps of the wavefront (as many as this launch holds),
  // else one step of a per-step order
  const int wlev = s->order_kind == MD_ORDER_WAVEFRONT ? (int)std::min<int64_t>(s->wlev, k_steps) : 1;
  if (s->order_dirty || wlev != s->order_wlev) {
    std::vector<uint32_t> ord;
    if (s->order_kind == MD_ORDER_WAVEFRONT) {
      ord = make_wavefront(g.S, wlev);
    } else {
      const std::vector<uint16_t> o =
          make_order(g.S, s->order_kind == MD_ORDER_DATAFLOW ? MD_ORDER_SWEEP : s->order_kind, s->order_seed);
      ord.assign(o.begin(), o.end());
    }
    HIPCHK(hipMemcpy(s->b.order, ord.data(), ord.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    s->order_dirty = false;
    s->order_wlev = wlev;
  }
  if (k_steps % wlev != 0) return fail(MD_EINVAL, "launch of %lld steps is not whole rounds of %d", (long long)k_steps, wlev);
  int64_t nsample = 0, first_j = 0;
  launch_samples(s, k_steps, &nsample, &first_j);
  const size_t ep = (size_t)std::max<int64_t>(nsample, 1) * g.S * s->nch * 3;
  const size_t ml = s->miglog_on ? (size_t)k_steps * g.S * 2 : 1;
  if (arena) {
    s->cur_epart = arena->take<double>(ep);
    s->cur_miglog = arena->take<uint32_t>(ml);
    if (!s->cur_epart || !s->cur_miglog) return fail(MD_EINVAL, "launch scratch exhausted");
  } else {
    // when they grow, sized for a launch of reserve_steps steps if that is more (at most
    // reserve_steps / every + 1 samples)
    const int64_t rk = std::max<int64_t>(k_steps, reserve_steps);
    if (ep > s->epart_cap) {
      const int64_t rs = s->every > 0 ? rk / s->every + 1 : 1;
      const size_t want = std::max(ep, (size_t)rs * g.S * s->nch * 3);
      dfree(s->d_epart);
      if ((rc = dalloc(&s->d_epart, want))) return rc;
      s->epart_cap = want;
    }
    if (ml > s->miglog_cap) {
      const size_t want = std::max(ml, s->miglog_on ? (size_t)rk * g.S * 2 : (size_t)1);
      dfree(s->d_miglog);
      if ((rc = dalloc(&s->d_miglog, want))) return rc;
      s->miglog_cap = want;
    }
    s->cur_epart = s->d_epart;
    s->cur_miglog = s->d_miglog;
  }
  if (s->miglog_on && launch_clear_u32(s->cur_miglog, (long long)ml, 0u, st)) return fail(MD_EHIP, "clear failed");
  // the launch's init kernel clears the error word and the pair counters
  std::memset(ra, 0, sizeof(*ra));
  ra->g = g;
  for (int p = 0; p < 2; p++) {
    ra->cells[p] = s->b.cells[p];
    ra->ncnt[p] = s->b.ncnt[p];
    ra->nin[p] = s->b.nin[p];
  }
  ra->cntA = s->b.cntA;
  ra->cntF = s->b.cntF;
  ra->epart = s->cur_epart;
  ra->miglog = s->miglog_on ? s->cur_miglog : nullptr;
  ra->migcum = s->b.migcum;
  ra->paircnt = s->b.paircnt;
  ra->err = s->b.err;
  ra->abort = s->b.abort;
  ra->order = s->b.order;
  ra->wlev = wlev;
  ra->t0 = s->t;
  ra->nsteps = (int)k_steps;
  ra->par0 = s->par;
  ra->first = s->first;
  ra->nch = s->nch;
  // finalise items: a quarter as many as force items under the dataflow scheduler (each
  // is short and every item pays a release and an acquire); as many with a fixed claim
  // order, whose tickets enumerate equal chunk counts for both phases
  ra->nchA = dataflow ? (int)finalise_items(s->nch) : s->nch;
  ra->every = (int)s->every;
  ra->count = s->count_pairs ? 1 : 0;
  ra->fail_at = s->fail_at;
  ra->ips = g.S * (s->nch + ra->nchA);
  if (s->thermo_T > 0.0) {
    if (s->order_kind != MD_ORDER_DATAFLOW)
      return fail(MD_EINVAL, "the thermostat runs with the dataflow scheduler only");
    if (!s->d_fbuf && (rc = dalloc(&s->d_fbuf, (size_t)g.ncell * 3 * CELL_CAP))) return rc;
    const size_t kp = (size_t)g.S * s->nch * 2;
    if (kp > s->kpart_cap) {
      dfree(s->d_kpart);
      if ((rc = dalloc(&s->d_kpart, kp))) return rc;
      s->kpart_cap = kp;
    }
    ra->thermo_T = s->thermo_T;
    ra->fbuf = s->d_fbuf;
    ra->kpart = s->d_kpart;
    ra->cntK = s->b.cntK;
    ra->ips = g.S * (2 * s->nch + ra->nchA);
  }
  *nsample_out = nsample;
  *first_j_out = first_j;
  return MD_OK;
}

// After a launch: error word w (gathered for all runs of the launch), energy samples,
// migration log, counters, step.
static int finish_run(md_sim* s, uint32_t w, int64_t k_steps, int64_t nsample, int64_t first_j) {
  const DGeom& g = s->g;
  if (w) return fail(err_status(w), "step at t=%lld: %s", (long long)s->t, err_text(w));
  if (nsample > 0) {
    std::vector<double> part((size_t)nsample * g.S * s->nch * 3);
    HIPCHK(hipMemcpy(part.data(), s->cur_epart, part.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t j = 0; j < nsample; j++) {
      double U = 0, K = 0, W = 0;
      const double* p = part.data() + (size_t)j * g.S * s->nch * 3;
      for (int64_t q = 0; q < (int64_t)g.S * s->nch; q++) {
        U += p[3 * q];
        K += p[3 * q + 1];
        W += p[3 * q + 2];
      }
      s->elog.push_back((double)((first_j + j) * s->every));
      s->elog.push_back(U);
      s->elog.push_back(K);
      s->elog.push_back(W);
    }
  }
  if (s->miglog_on) {
    const size_t off = s->miglog.size();
    s->miglog.resize(off + (size_t)k_steps * g.S * 2);
    HIPCHK(hipMemcpy(s->miglog.data() + off, s->cur_miglog, (size_t)k_steps * g.S * 2 * sizeof(uint32_t),
                     hipMemcpyDeviceToHost));
    s->miglog_steps += k_steps;
  }
  if (s->count_pairs) {
    unsigned long long pc[2];
    HIPCHK(hipMemcpy(pc, s->b.paircnt, sizeof(pc), hipMemcpyDeviceToHost));
    s->cand += (int64_t)pc[0];
    s->inr += (int64_t)pc[1];
    s->counted += s->n * k_steps;
  }
  s->t += k_steps;
  s->par = (int)((s->par + k_steps) & 1);
  s->first = 0;
  return MD_OK;
}

// Cost of a cell in atom equivalents when the slices are split among the XCD work queues:
// every cell is staged and walked (and its neighbourhood counted) whether or not it holds
// atoms, so sparse slices cost more than their atoms alone.
constexpr double QUEUE_CELL_COST = 4.0;

// Work-queue ranges of s for the next md_step: one contiguous range of slices per XCD,
// each of at least 3 slices, with boundaries where the cumulative cost (atoms plus
// QUEUE_CELL_COST per cell) is closest to equal shares.  One queue for the device when the
// option is off, the claim order is fixed, the GPU has one XCD, or there are fewer than 3
// slices per XCD.
static int plan_queues(md_sim* s) {
  const DGeom& g = s->g;
  const int S = g.S;
  s->nq = 1;
  s->xfirst[0] = 0;
  for (int x = 1; x <= MAX_XQ; x++) s->xfirst[x] = S;
  const int nx = s->nxcc;
  if (!s->xcd_queues || nx <= 1 || s->order_kind != MD_ORDER_DATAFLOW || S < 3 * nx) return MD_OK;
  if (launch_slice_counts(g, s->b.ncnt[s->par], s->b.scount, s->stream)) return fail(MD_EHIP, "slice counts failed");
  std::vector<unsigned long long> cnt((size_t)S);
  HIPCHK(hipMemcpyAsync(cnt.data(), s->b.scount, (size_t)S * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                        s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  std::vector<double> cum((size_t)S + 1, 0.0);
  for (int i = 0; i < S; i++) cum[(size_t)i + 1] = cum[(size_t)i] + (double)cnt[(size_t)i] + QUEUE_CELL_COST * g.cps;
  const double W = cum[(size_t)S];
  for (int x = 1; x < nx; x++) {
    const double target = W * x / nx;
    const int lo = s->xfirst[x - 1] + 3, hi = S - 3 * (nx - x);
    int best = lo;
    for (int e = lo; e <= hi; e++)
      if (std::fabs(cum[(size_t)e] - target) < std::fabs(cum[(size_t)best] - target)) best = e;
    s->xfirst[x] = best;
  }
  s->nq = nx;
  return MD_OK;
}

// Launch k[r] steps of every simulation in `sims` (all of one precision) as one
// persistent kernel.  status[r] receives each run's own result.
static int packed_launch(std::vector<md_sim*>& sims, std::vector<int64_t>& ksteps, LaunchScratch& ls,
                         hipStream_t st, int64_t grid_override, int64_t watchdog_ms, int* last_grid,
                         std::vector<int>& status, double* kernel_seconds = nullptr,
                         md_sim* trace_owner = nullptr, uint32_t launch_index = 0, Carve* arena = nullptr,
                         int64_t reserve_rounds = 0) {
  const size_t R = sims.size();
  status.assign(R, MD_OK);
  if (R == 0) return MD_OK;
  // runs sorted by steps (descending): the runs active in round k are a prefix
  std::vector<size_t> idx(R);
  for (size_t r = 0; r < R; r++) idx[r] = r;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return ksteps[a] > ksteps[b]; });
  const int64_t nrounds = ksteps[idx[0]];
  if (nrounds <= 0) return MD_OK;
  // launch-wide buffers: the caller's scratch pieces, or ls (grown as needed)
  RunArgs* d_runs;
  long long *d_run_prefix, *d_round_base;
  int* d_round_active;
  unsigned long long *d_ticket, *d_q_tail;
  uint32_t *d_launch_err, *d_errs;
  int rc;
  if (arena) {
    d_runs = arena->take<RunArgs>(R);
    d_run_prefix = arena->take<long long>(R + 1);
    d_round_base = arena->take<long long>((size_t)nrounds + 1);
    d_round_active = arena->take<int>((size_t)nrounds + 1);
    d_ticket = arena->take<unsigned long long>((size_t)MAX_XQ * XQ_STRIDE);
    d_q_tail = arena->take<unsigned long long>((size_t)MAX_XQ * XQ_STRIDE);
    d_launch_err = arena->take<uint32_t>(1);
    d_errs = arena->take<uint32_t>(R);
    if (!d_runs || !d_run_prefix || !d_round_base || !d_round_active || !d_ticket || !d_q_tail || !d_launch_err ||
        !d_errs)
      return fail(MD_EINVAL, "launch scratch exhausted");
  } else {
    // when they grow, the round tables and the queue (below) are sized for reserve_rounds
    // rounds if that is more, so that a longer launch later does not allocate again
    if ((rc = ls.reserve(R, (size_t)std::max<int64_t>(nrounds, reserve_rounds)))) return rc;
    d_runs = ls.d_runs;
    d_run_prefix = ls.d_run_prefix;
    d_round_base = ls.d_round_base;
    d_round_active = ls.d_round_active;
    d_ticket = ls.d_ticket;
    d_q_tail = ls.d_q_tail;
    d_launch_err = ls.d_launch_err;
    d_errs = ls.d_errs;
  }
  std::vector<RunArgs> ra(R);
  std::vector<int64_t> nsample(R), first_j(R);
  std::vector<long long> prefix(R + 1, 0);
  int max_slices = 1;
  const int prec = sims[idx[0]]->prec;
  const int mode = sims[idx[0]]->order_kind == MD_ORDER_DATAFLOW ? 0 : 1;
  for (size_t q = 0; q < R; q++) {
    md_sim* s = sims[idx[q]];
    if ((rc = prepare_run(s, ksteps[idx[q]], mode == 0, st, &ra[q], &nsample[idx[q]], &first_j[idx[q]], arena,
                          reserve_rounds)))
      return rc;
    prefix[q + 1] = prefix[q] + ra[q].ips;
    max_slices = std::max(max_slices, s->g.S);
  }
  // kernel variant: pair counting (or fault injection) > energy samples > plain steps
  int kind = 0, nvt = 0;
  for (size_t q = 0; q < R; q++) {
    if (ra[q].count || ra[q].fail_at >= 0) kind = 2;
    else if (nsample[idx[q]] > 0) kind = std::max(kind, 1);
    if (ra[q].thermo_T > 0.0) nvt = 1;
  }
  const int grid = grid_size(prec, kind, nvt, grid_override);
  // work queues: one per XCD for a single run that planned them (dataflow only), else one;
  // workgroups are dealt to the XCDs in turn, so every queue has workers once the grid
  // holds at least two workgroups per queue
  int nq = 1;
  if (mode == 0 && R == 1 && sims[0]->nq > 1 && grid >= 2 * sims[0]->nq) nq = sims[0]->nq;
  if (R == 1 && nq == 1 && sims[0]->nq > 1) {  // planned, but not possible with this grid
    sims[0]->nq = 1;
    for (int x = 1; x <= MAX_XQ; x++) sims[0]->xfirst[x] = sims[0]->g.S;
  }
  std::vector<long long> qtotal(MAX_XQ, 0), qfill(MAX_XQ, 0);
  for (size_t q = 0; q < R; q++) {
    md_sim* s = sims[idx[q]];
    for (int x = 0; x <= MAX_XQ; x++) ra[q].xfirst[x] = nq > 1 ? s->xfirst[x] : (x == 0 ? 0 : s->g.S);
    const long long per_slice = ra[q].ips / s->g.S;  // items of one slice per step
    for (int x = 0; x < nq; x++) {
      const long long nsl = ra[q].xfirst[x + 1] - ra[q].xfirst[x];
      ra[q].q0[x] = qfill[(size_t)x];
      if (ksteps[idx[q]] <= 0) continue;  // a run without steps here queues nothing
      qfill[(size_t)x] += nsl * ra[q].nch;
      qtotal[(size_t)x] += ksteps[idx[q]] * nsl * per_slice;
    }
  }
  // tickets are dealt round by round; a round is one step of every active run, or the
  // wlev steps of the one run of a wavefront launch
  const int spr = (mode == 1 && R == 1) ? ra[0].wlev : 1;
  const int64_t nrounds_d = nrounds / spr;
  if (spr > 1)
    for (size_t q = 0; q <= R; q++) prefix[q] *= spr;
  std::vector<long long> rb((size_t)nrounds_d + 1, 0);
  std::vector<int> act((size_t)nrounds_d + 1, 0);
  size_t a = R;
  for (int64_t k = 0; k < nrounds_d; k++) {
    while (a > 0 && ksteps[idx[a - 1]] <= k * spr) a--;
    act[(size_t)k] = (int)a;
    rb[(size_t)k + 1] = rb[(size_t)k] + prefix[a];
  }
  HIPCHK(hipMemcpy(d_runs, ra.data(), R * sizeof(RunArgs), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d_run_prefix, prefix.data(), prefix.size() * sizeof(long long), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d_round_base, rb.data(), rb.size() * sizeof(long long), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d_round_active, act.data(), act.size() * sizeof(int), hipMemcpyHostToDevice));
  const size_t total = (size_t)rb[(size_t)nrounds_d];
  if (nrounds >= (1 << 19)) return fail(MD_EINVAL, "too many steps in one launch");
  unsigned long long* d_q = nullptr;
  if (mode == 0) {
    if (arena) {
      if (!(d_q = arena->take<unsigned long long>(total))) return fail(MD_EINVAL, "launch scratch exhausted");
    } else {
      if (total > ls.q_cap) {
        // items of a round with every run active, times the rounds reserved beyond this launch
        const size_t per_round = nrounds_d > 0 ? (size_t)(rb[1] - rb[0]) : 0;
        const size_t want = total + (size_t)std::max<int64_t>(reserve_rounds - nrounds_d, 0) * per_round;
        dfree(ls.d_q);
        if ((rc = dalloc(&ls.d_q, want))) return rc;
        ls.q_cap = want;
      }
      d_q = ls.d_q;
    }
    // slots start empty (the top bit marks a pushed item)
    if (launch_clear_u32(reinterpret_cast<uint32_t*>(d_q), (long long)(2 * total), 0u, st))
      return fail(MD_EHIP, "clear failed");
  }
  LaunchArgs la{};
  la.runs = d_runs;
  la.nruns = (int)R;
  la.nrounds = (int)nrounds_d;
  la.round_base = d_round_base;
  la.round_active = d_round_active;
  la.run_prefix = d_run_prefix;
  la.ticket = d_ticket;
  la.watchdog_ticks = watchdog_ticks(watchdog_ms);
  la.trace = nullptr;
  la.launch_index = launch_index;
  la.mode = mode;
  la.q = d_q;
  la.q_tail = d_q_tail;
  la.launch_err = d_launch_err;
  la.total = (long long)total;
  la.nq = nq;
  la.qoff[0] = 0;
  for (int x = 0; x < MAX_XQ; x++) {
    la.qoff[x + 1] = x < nq ? la.qoff[x] + qtotal[(size_t)x] : la.qoff[x];
    la.prefill[x] = qfill[(size_t)x];
  }
  if (nq == 1) la.qoff[1] = (long long)total;
  for (int x = nq + 1; x <= MAX_XQ; x++) la.qoff[x] = la.qoff[nq];
  if (mode == 0 && la.qoff[nq] != (long long)total)
    return fail(MD_EINVAL, "work queues hold %lld items, the launch %lld", la.qoff[nq], (long long)total);
  long long prefill = 0;
  for (size_t q = 0; q < R; q++) prefill += (long long)ra[q].g.S * ra[q].nch;
  if (trace_owner && trace_owner->trace_on) {
    if (total > trace_owner->trace_cap) {
      dfree(trace_owner->d_trace);
      if ((rc = dalloc(&trace_owner->d_trace, total))) return rc;
      trace_owner->trace_cap = total;
    }
    if (launch_clear_u32(reinterpret_cast<uint32_t*>(trace_owner->d_trace),
                         (long long)(total * sizeof(TraceRec) / 4), 0u, st))
      return fail(MD_EHIP, "clear failed");
    la.trace = trace_owner->d_trace;
  }
  if (launch_init(la, std::max<long long>(prefill, max_slices), st)) return fail(MD_EHIP, "init failed");
  if (last_grid) *last_grid = grid;
  if (kernel_seconds && !ls.ev[0]) {
    HIPCHK(hipEventCreate(&ls.ev[0]));
    HIPCHK(hipEventCreate(&ls.ev[1]));
  }
  if (kernel_seconds) HIPCHK(hipEventRecord(ls.ev[0], st));
  if (launch_persistent(la, prec, kind, nvt, grid, st)) return fail(MD_EHIP, "persistent launch failed");
  if (kernel_seconds) HIPCHK(hipEventRecord(ls.ev[1], st));
  HIPCHK(hipStreamSynchronize(st));
  if (kernel_seconds) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ls.ev[0], ls.ev[1]));
    *kernel_seconds = 1e-3 * (double)ms;
  }
  if (la.trace) {
    const size_t off = trace_owner->trace.size();
    trace_owner->trace.resize(off + total);
    HIPCHK(hipMemcpy(trace_owner->trace.data() + off, la.trace, total * sizeof(TraceRec), hipMemcpyDeviceToHost));
  }
  uint32_t lerr = 0;
  HIPCHK(hipMemcpy(&lerr, d_launch_err, sizeof(uint32_t), hipMemcpyDeviceToHost));
  if (lerr) {
    for (size_t r = 0; r < R; r++)
      status[r] = (lerr & ERR_BADINPUT) ? fail(MD_EHIP, "a work queue overflowed (internal error)")
                                        : fail(MD_EWATCHDOG, "a work-queue wait exceeded the watchdog");
    return MD_OK;
  }
  // every run's error word with one copy (ra and d_runs are in sorted order idx)
  // (the launch stream is non-blocking: the copy goes on it, then the stream is waited for)
  if (launch_gather_errors(d_runs, (int)R, d_errs, st)) return fail(MD_EHIP, "error gather failed");
  std::vector<uint32_t> errs(R, 0u);
  HIPCHK(hipMemcpyAsync(errs.data(), d_errs, R * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (size_t q = 0; q < R; q++) {
    const size_t r = idx[q];
    status[r] = finish_run(sims[r], errs[q], ksteps[r], nsample[r], first_j[r]);
  }
  return MD_OK;
}

extern "C" int md_step(md_sim* s, int64_t nsteps) {
  if (!s) return fail(MD_EINVAL, "sim is NULL");
  if (!s->loaded) return fail(MD_ESTATE, "md_step before md_load");
  if (s->poisoned) return fail(MD_ESTATE, "handle poisoned by an earlier failure");
  if (nsteps < 0) return fail(MD_EINVAL, "nsteps must be >= 0");
  s->elog.clear();
  s->miglog.clear();
  s->miglog_steps = 0;
  s->cand = s->inr = s->counted = 0;
  s->last_kernel_seconds = 0;
  s->last_launches = 0;
  s->trace.clear();
  const auto t0 = std::chrono::steady_clock::now();
  if (nsteps > 0) {
    const int prc = plan_queues(s);
    if (prc) return prc;
  }
  int64_t left = nsteps;
  std::vector<md_sim*> one(1, s);
  std::vector<int64_t> ks(1);
  std::vector<int> st;
  // the launch buffers, when they grow, are sized for the longest launch this run may make
  // (its steps-per-launch cap; at most a 64 MB work queue), so that stepping on after a
  // shorter launch does not allocate
  const int64_t queue_bytes_per_step = 8ll * s->g.S * (2ll * s->nch + finalise_items(s->nch));
  const int64_t reserve = std::min<int64_t>(s->max_steps_per_launch,
                                            std::max<int64_t>(1, (64ll << 20) / queue_bytes_per_step));
  while (left > 0) {
    ks[0] = std::min(left, s->max_steps_per_launch);
    // a wavefront launch holds whole rounds of wlev steps; a shorter rest runs alone
    if (s->order_kind == MD_ORDER_WAVEFRONT && ks[0] >= s->wlev) ks[0] -= ks[0] % s->wlev;
    double ksec = 0;
    int rc = packed_launch(one, ks, *s->ls, s->stream, s->grid_override, s->watchdog_ms, &s->last_grid, st,
                           &ksec, s, (uint32_t)s->last_launches, nullptr, reserve);
    s->last_kernel_seconds += ksec;
    s->last_launches++;
    if (!rc) rc = st[0];
    if (rc) {
      s->poisoned = true;
      return rc;
    }
    left -= ks[0];
  }
  s->last_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return MD_OK;
}

// Scratch bytes of one launch of k steps of s, carved in the order packed_launch and
// prepare_run take them (each piece rounded up to 256 bytes).
static size_t noalloc_launch_bytes(const md_sim* s, int64_t k) {
  const DGeom& g = s->g;
  const bool dataflow = s->order_kind == MD_ORDER_DATAFLOW;
  int64_t nsample = 0, first_j = 0;
  launch_samples(s, k, &nsample, &first_j);
  size_t b = round256(sizeof(RunArgs)) + round256(2 * sizeof(long long));
  b += round256((size_t)(k + 1) * sizeof(long long)) + round256((size_t)(k + 1) * sizeof(int));
  b += 2 * round256((size_t)MAX_XQ * XQ_STRIDE * sizeof(unsigned long long)) + 2 * round256(sizeof(uint32_t));
  b += round256((size_t)std::max<int64_t>(nsample, 1) * g.S * s->nch * 3 * sizeof(double));
  b += round256((s->miglog_on ? (size_t)k * g.S * 2 : 1) * sizeof(uint32_t));
  if (dataflow) {
    const size_t ips = (size_t)g.S * (size_t)(s->nch + finalise_items(s->nch));
    b += round256((size_t)k * ips * sizeof(unsigned long long));
  }
  return b;
}

extern "C" int md_step_noalloc(md_sim* s, int64_t nsteps) {
  if (!s) return fail(MD_EINVAL, "sim is NULL");
  if (!s->loaded) return fail(MD_ESTATE, "md_step_noalloc before md_load");
  if (s->poisoned) return fail(MD_ESTATE, "handle poisoned by an earlier failure");
  if (nsteps < 0) return fail(MD_EINVAL, "nsteps must be >= 0");
  if (s->thermo_T > 0.0)
    return fail(MD_EINVAL, "md_step_noalloc does not run the thermostat (its force buffer is allocated)");
  if (s->trace_on) return fail(MD_EINVAL, "md_step_noalloc does not record traces (MD_OPT_TRACE)");
  unsigned char* base = s->dev >= 0 && s->dev < SCRATCH_MAX_DEVICES ? g_scratch_dev[s->dev] : nullptr;
  if (!base) return fail(MD_EHIP, "no launch scratch on device %d", s->dev);
  const size_t one = noalloc_launch_bytes(s, 1);
  if (one > (size_t)MD_NOALLOC_SCRATCH_BYTES)
    return fail(MD_EINVAL, "one step of this system needs %zu bytes of launch scratch; md_step_noalloc has %zu",
                one, (size_t)MD_NOALLOC_SCRATCH_BYTES);
  s->elog.clear();
  s->miglog.clear();
  s->miglog_steps = 0;
  s->cand = s->inr = s->counted = 0;
  s->last_kernel_seconds = 0;
  s->last_launches = 0;
  s->trace.clear();
  const auto t0 = std::chrono::steady_clock::now();
  if (nsteps > 0) {
    const int prc = plan_queues(s);
    if (prc) return prc;
  }
  int64_t left = nsteps;
  std::vector<md_sim*> sims(1, s);
  std::vector<int64_t> ks(1);
  std::vector<int> st;
  while (left > 0) {
    // the longest launch (within the step cap) whose pieces fit the scratch
    int64_t lo = 1, hi = std::min(left, s->max_steps_per_launch);
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (noalloc_launch_bytes(s, mid) <= (size_t)MD_NOALLOC_SCRATCH_BYTES) lo = mid;
      else hi = mid - 1;
    }
    if (s->order_kind == MD_ORDER_WAVEFRONT && lo >= s->wlev) lo -= lo % s->wlev;
    ks[0] = lo;
    Carve arena{base, (size_t)MD_NOALLOC_SCRATCH_BYTES, 0};
    int rc = packed_launch(sims, ks, *s->ls, s->stream, s->grid_override, s->watchdog_ms, &s->last_grid, st,
                           nullptr, nullptr, (uint32_t)s->last_launches, &arena);
    s->last_launches++;
    if (!rc) rc = st[0];
    if (rc) {
      s->poisoned = true;
      return rc;
    }
    left -= ks[0];
  }
  s->last_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return MD_OK;
}

// ---------------------------------------------------------------------------
// synchronous read-back
// ---------------------------------------------------------------------------
static int sync_pass(md_sim* s, double* hpos, double* hvel, double* hforce, double* U, double* K, double* W) {
  const DGeom& g = s->g;
  hipStream_t st = s->stream;
  const int blocks = sync_blocks(g);
  double* epart = nullptr;
  double *dpos = nullptr, *dvel = nullptr, *dfor = nullptr;
  int rc = dalloc(&epart, (size_t)blocks * 3);
  if (rc) return rc;
  const size_t nn = (size_t)std::max<int64_t>(s->n, 1) * 3;
  if ((hpos && (rc = dalloc(&dpos, nn))) || (hvel && (rc = dalloc(&dvel, nn))) ||
      (hforce && (rc = dalloc(&dfor, nn)))) {
    dfree(epart); dfree(dpos); dfree(dvel); dfree(dfor);
    return rc;
  }
  int l = launch_sync(g, s->b.cells[s->par], s->b.ncnt[s->par], s->first, dpos, dvel, dfor, epart,
                      s->b.err, st);
  hipError_t e = hipStreamSynchronize(st);
  rc = MD_OK;
  if (l || e != hipSuccess) rc = fail(MD_EHIP, "sync pass failed: %s", hipGetErrorString(e));
  if (!rc) {
    std::vector<double> part((size_t)blocks * 3);
    if (hipMemcpy(part.data(), epart, part.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      rc = fail(MD_EHIP, "copy failed");
    double u = 0, k = 0, w = 0;
    for (int b = 0; b < blocks; b++) {
      u += part[3 * b];
      k += part[3 * b + 1];
      w += part[3 * b + 2];
    }
    if (U) *U = u;
    if (K) *K = k;
    if (W) *W = w;
    const size_t bytes = sizeof(double) * 3 * (size_t)s->n;
    if (!rc && s->n > 0) {
      if (hpos && hipMemcpy(hpos, dpos, bytes, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(MD_EHIP, "copy failed");
      if (hvel && hipMemcpy(hvel, dvel, bytes, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(MD_EHIP, "copy failed");
      if (hforce && hipMemcpy(hforce, dfor, bytes, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(MD_EHIP, "copy failed");
    }
  }
  dfree(epart); dfree(dpos); dfree(dvel); dfree(dfor);
  return rc;
}

extern "C" int md_energy_virial(md_sim* s, double* U, double* K, double* W) {
  if (!s) return fail(MD_EINVAL, "sim is NULL");
  if (!s->loaded) return fail(MD_ESTATE, "no state loaded");
  if (s->poisoned) return fail(MD_ESTATE, "handle poisoned by an earlier failure");
  return sync_pass(s, nullptr, nullptr, nullptr, U, K, W);
}

extern "C" int md_get_state(md_sim* s, double* pos, double* vel, double* force) {
  if (!s) return fail(MD_EINVAL, "sim is NULL");
  if (!s->loaded) return fail(MD_ESTATE, "no state loaded");
  if (s->poisoned) return fail(MD_ESTATE, "handle poisoned by an earlier failure; reload a saved state");
  return sync_pass(s, pos, vel, force, nullptr, nullptr, nullptr);
}

extern "C" int md_get_cells(md_sim* s, int64_t* cell) {
  if (!s || (!cell && s->n > 0)) return fail(MD_EINVAL, "bad arguments");
  if (!s->loaded || s->poisoned) return fail(MD_ESTATE, "no valid state");
  if (s->n == 0) return MD_OK;
  long long* d = nullptr;
  int rc = dalloc(&d, (size_t)s->n);
  if (rc) return rc;
  int l = launch_cells_of(s->g, s->b.ncnt[s->par], s->b.cells[s->par], d, s->stream);
  hipError_t e = hipStreamSynchronize(s->stream);
  if (!l && e == hipSuccess)
    e = hipMemcpy(cell, d, sizeof(long long) * (size_t)s->n, hipMemcpyDeviceToHost);
  dfree(d);
  if (l || e != hipSuccess) return fail(MD_EHIP, "cell read-back failed");
  return MD_OK;
}

extern "C" int md_get_slice_counts(md_sim* s, int64_t* counts) {
  if (!s || !counts) return fail(MD_EINVAL, "bad arguments");
  if (!s->loaded || s->poisoned) return fail(MD_ESTATE, "no valid state");
  unsigned long long* d = nullptr;
  int rc = dalloc(&d, (size_t)s->g.S);
  if (rc) return rc;
  int l = launch_slice_counts(s->g, s->b.ncnt[s->par], d, s->stream);
  hipError_t e = hipStreamSynchronize(s->stream);
  std::vector<unsigned long long> h((size_t)s->g.S);
  if (!l && e == hipSuccess) e = hipMemcpy(h.data(), d, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
  dfree(d);
  if (l || e != hipSuccess) return fail(MD_EHIP, "slice count read-back failed");
  for (int i = 0; i < s->g.S; i++) counts[i] = (int64_t)h[i];
  return MD_OK;
}

extern "C" int md_get_energy_log(md_sim* s, int64_t cap_rows, double* rows, int64_t* count) {
  if (!s || !count || cap_rows < 0 || (cap_rows > 0 && !rows)) return fail(MD_EINVAL, "bad arguments");
  const int64_t have = (int64_t)s->elog.size() / 4;
  const int64_t m = std::min(have, cap_rows);
  if (m > 0) std::memcpy(rows, s->elog.data(), sizeof(double) * 4 * (size_t)m);
  *count = have;
  return MD_OK;
}

extern "C" int md_get_migration_log(md_sim* s, int64_t cap_steps, int32_t* log, int64_t* steps) {
  if (!s || !steps || cap_steps < 0 || (cap_steps > 0 && !log)) return fail(MD_EINVAL, "bad arguments");
  const int64_t m = std::min(s->miglog_steps, cap_steps);
  if (m > 0) std::memcpy(log, s->miglog.data(), sizeof(int32_t) * 2 * s->g.S * (size_t)m);
  *steps = s->miglog_steps;
  return MD_OK;
}

extern "C" int md_get_trace(md_sim* s, int64_t cap, md_trace_rec* out, int64_t* count, double* hz) {
  static_assert(sizeof(md_trace_rec) == sizeof(TraceRec), "trace record layout");
  if (!s || !count || cap < 0 || (cap > 0 && !out)) return fail(MD_EINVAL, "bad arguments");
  const int64_t have = (int64_t)s->trace.size();
  const int64_t m = std::min(have, cap);
  if (m > 0) std::memcpy(out, s->trace.data(), sizeof(TraceRec) * (size_t)m);
  *count = have;
  if (hz) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      khz = 100000;
    *hz = 1e3 * khz;
  }
  return MD_OK;
}

extern "C" int md_get_stats(md_sim* s, md_stats* out) {
  if (!s || !out) return fail(MD_EINVAL, "bad arguments");
  std::memset(out, 0, sizeof(*out));
  out->step = s->t;
  out->n = s->n;
  out->slices = s->g.S;
  out->ncx = s->g.ncx;
  for (int d = 0; d < 3; d++) out->grid[d] = s->g.G[d];
  out->cell_capacity = s->g.cap;
  out->ncell = s->g.ncell;
  if (s->loaded) {
    std::vector<unsigned long long> m((size_t)2 * s->g.S);
    if (hipMemcpy(m.data(), s->b.migcum, m.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) == hipSuccess) {
      for (int i = 0; i < s->g.S; i++) {
        out->migrations_left += (int64_t)m[2 * i];
        out->migrations_right += (int64_t)m[2 * i + 1];
      }
    }
  }
  out->candidates = s->cand;
  out->in_range = s->inr;
  out->counted_steps = s->counted;
  out->last_step_seconds = s->last_seconds;
  out->last_kernel_seconds = s->last_kernel_seconds;
  out->last_launches = s->last_launches;
  out->persistent_grid = s->last_grid;
  out->chunks_per_slice = s->nch;
  out->precision = s->prec;
  out->poisoned = s->poisoned ? 1 : 0;
  out->work_queues = s->nq;
  static_assert(MAX_XQ + 1 <= 9, "md_stats.queue_first holds MAX_XQ + 1 entries");
  for (int x = 0; x < 9; x++) out->queue_first[x] = x <= MAX_XQ ? s->xfirst[x] : s->g.S;
  return MD_OK;
}

// ---------------------------------------------------------------------------
// serving: continuous batching of independent runs
// ---------------------------------------------------------------------------
namespace {

struct ServedRun {
  uint64_t ticket = 0;
  md_run_desc d{};
  std::vector<double> pos, vel;  // input copies, dropped once on the device
  int64_t fp = 0;                // device bytes while resident
  md_sim* sim = nullptr;
  int status = MD_PENDING;
  bool polled = false;
  md_result res{};
  std::vector<double> out_pos, out_vel;
  std::vector<double> sample_t, sample_e;  // energy samples: step, (U + K) / n
};

double drift_slope(const std::vector<double>& ts, const std::vector<double>& es) {
  const size_t m = ts.size();
  if (m < 2) return 0.0;
  double mt = 0, me = 0;
  for (size_t i = 0; i < m; i++) {
    mt += ts[i];
    me += es[i];
  }
  mt /= (double)m;
  me /= (double)m;
  double sxy = 0, sxx = 0;
  for (size_t i = 0; i < m; i++) {
    sxy += (ts[i] - mt) * (es[i] - me);
    sxx += (ts[i] - mt) * (ts[i] - mt);
  }
  return sxx > 0 ? sxy / sxx : 0.0;
}

}  // namespace

struct md_server {
  size_t budget = 0;
  int max_runs = 1;
  int quantum = 0;
  int flags = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<ServedRun>> queue;
  std::vector<std::shared_ptr<ServedRun>> running;
  std::map<uint64_t, std::shared_ptr<ServedRun>> runs;
  int64_t in_use = 0, launches = 0, ndone = 0;
  // seconds the server thread spent admitting runs, in packed launches, completing runs
  // (read-back and release) and waiting for work
  double t_admit = 0, t_launch = 0, t_finish = 0, t_idle = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread th;
  hipStream_t stream = nullptr;
  LaunchScratch ls;
  std::chrono::steady_clock::time_point origin = std::chrono::steady_clock::now();
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - origin).count();
  }
};

static void finish_served(md_server* sv, const std::shared_ptr<ServedRun>& r, int status) {
  if (r->sim) {
    md_free(r->sim);
    r->sim = nullptr;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  r->res.status = status;
  r->res.t_done = sv->now();
  r->status = status;
  sv->in_use -= r->fp;
  sv->ndone++;
  sv->running.erase(std::remove(sv->running.begin(), sv->running.end(), r), sv->running.end());
}

// Bring an admitted run onto the device: geometry, binning, energy at t = 0.

static int admit_served(md_server* sv, ServedRun& r) {
  if (sv->flags & MD_SERVER_FAKE_EXECUTOR) return MD_OK;
  md_sim* s = nullptr;
  int rc = md_init(r.d.box, r.d.slices, r.d.rc, r.d.dt, r.d.precision, &s);
  if (rc) return rc;
  r.sim = s;
  // served runs are small: short work items keep each step's critical path short
  if ((rc = md_set_option(s, MD_OPT_CHUNK_CELLS, served_chunk_cells(s->g)))) return rc;
  if ((rc = md_set_stream(s, sv->stream))) return rc;
  if ((rc = md_load(s, r.d.n, r.pos.data(), r.vel.data()))) return rc;
  // energy samples every energy_every steps are taken inside the packed launches (the
  // energy-sampling kernel variant), t = 0 among them; t = steps by the read-back at the end
  if (r.d.energy_every > 0 && (rc = md_set_option(s, MD_OPT_ENERGY_EVERY, r.d.energy_every))) return rc;
  double U, K, W;
  if ((rc = md_energy_virial(s, &U, &K, &W))) return rc;
  r.res.U0 = U;
  r.res.K0 = K;
  r.res.W0 = W;
  if (r.d.energy_every <= 0) {
    r.sample_t.push_back(0.0);
    r.sample_e.push_back((U + K) / (double)std::max<int64_t>(r.d.n, 1));
  }
  std::vector<double>().swap(r.pos);
  std::vector<double>().swap(r.vel);
  return MD_OK;
}

// Last step reached: energy at t = steps, drift, optional final state.
static int complete_served(md_server* sv, ServedRun& r) {
  (void)sv;
  r.res.steps_done = r.d.steps;
  if (sv->flags & MD_SERVER_FAKE_EXECUTOR) return MD_OK;
  md_sim* s = r.sim;
  double U, K, W;
  int rc = md_energy_virial(s, &U, &K, &W);
  if (rc) return rc;
  r.res.U1 = U;
  r.res.K1 = K;
  r.res.W1 = W;
  std::vector<double> ts = r.sample_t, es = r.sample_e;
  const double n = (double)std::max<int64_t>(r.d.n, 1);
  for (size_t j = 0; j + 3 < s->elog.size(); j += 4) {  // in-launch samples: (t, U, K, W)
    ts.push_back(s->elog[j]);
    es.push_back((s->elog[j + 1] + s->elog[j + 2]) / n);
  }
  ts.push_back((double)r.d.steps);
  es.push_back((U + K) / n);
  r.res.drift_per_atom_step = drift_slope(ts, es);
  if (r.d.keep_state) {
    r.out_pos.resize((size_t)3 * r.d.n);
    r.out_vel.resize((size_t)3 * r.d.n);
    if ((rc = md_get_state(s, r.out_pos.data(), r.out_vel.data(), nullptr))) return rc;
  }
  return MD_OK;
}

static void server_loop(md_server* sv) {
  const bool fake = (sv->flags & MD_SERVER_FAKE_EXECUTOR) != 0;
  if (!fake) (void)hipSetDevice(sv->device);
  std::vector<int64_t> done_steps;
  auto clock = [] { return std::chrono::steady_clock::now(); };
  auto secs = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
    return std::chrono::duration<double>(b - a).count();
  };
  while (true) {
    std::vector<std::shared_ptr<ServedRun>> admit;
    const auto t_wait = clock();
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      while (true) {
        if (sv->stop) return;
        // first come, first served: the head of the queue is admitted when its footprint
        // fits next to the resident runs and a slot is free; nobody overtakes it
        while (!sv->queue.empty() && (int)(sv->running.size() + admit.size()) < sv->max_runs &&
               sv->in_use + sv->queue.front()->fp <= (int64_t)sv->budget) {
          std::shared_ptr<ServedRun> r = sv->queue.front();
          sv->queue.pop_front();
          sv->in_use += r->fp;
          r->res.t_admit = sv->now();
          admit.push_back(r);
        }
        if (!sv->running.empty() || !admit.empty()) break;
        sv->cv.wait_for(lk, std::chrono::milliseconds(20));
      }
      for (auto& r : admit) sv->running.push_back(r);
    }
    const auto t_adm = clock();
    for (auto& r : admit) {
      int rc = admit_served(sv, *r);
      if (rc) finish_served(sv, r, rc);
    }
    {
      const auto t_end = clock();
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->t_idle += secs(t_wait, t_adm);
      sv->t_admit += secs(t_adm, t_end);
    }
    std::vector<std::shared_ptr<ServedRun>> cur;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      cur = sv->running;
    }
    if (cur.empty()) continue;
    // one bounded launch per precision over every resident run
    for (int prec = 0; prec < 2; prec++) {
      std::vector<std::shared_ptr<ServedRun>> grp;
      std::vector<md_sim*> sims;
      std::vector<int64_t> ks;
      for (auto& r : cur) {
        if (r->d.precision != prec) continue;
        const int64_t t = fake ? r->res.steps_done : r->sim->t;
        const int64_t left = r->d.steps - t;
        if (left <= 0) continue;
        const int64_t q = sv->quantum > 0 ? sv->quantum : SERVED_QUANTUM;
        const int64_t k = std::min(left, q);
        grp.push_back(r);
        sims.push_back(r->sim);
        ks.push_back(k);
      }
      if (grp.empty()) continue;
      std::vector<int> st(grp.size(), MD_OK);
      int rc = MD_OK;
      const auto t_l0 = clock();
      if (fake) {
        int64_t work = 0;
        for (size_t i = 0; i < grp.size(); i++) {
          work = std::max<int64_t>(work, grp[i]->d.n * ks[i]);
          grp[i]->res.steps_done += ks[i];
        }
        std::this_thread::sleep_for(std::chrono::microseconds(100 + work / 20000));
      } else {
        rc = packed_launch(sims, ks, sv->ls, sv->stream, 0, 20000, nullptr, st);
      }
      const auto t_l1 = clock();
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->launches++;
        sv->t_launch += secs(t_l0, t_l1);
      }
      for (size_t i = 0; i < grp.size(); i++) {
        const int s = rc ? rc : st[i];
        if (s) {
          finish_served(sv, grp[i], s);
          continue;
        }
        const int64_t t = fake ? grp[i]->res.steps_done : grp[i]->sim->t;
        if (t >= grp[i]->d.steps) finish_served(sv, grp[i], complete_served(sv, *grp[i]));
      }
      {
        const auto t_f = clock();
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->t_finish += secs(t_l1, t_f);
      }
    }
  }
}

extern "C" int md_server_create_ex(size_t hbm_budget_bytes, int max_runs, int quantum_steps, int flags,
                                   md_server** out) {
  if (!out) return fail(MD_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes == 0 || max_runs < 1 || quantum_steps < 0) return fail(MD_EINVAL, "bad server limits");
  LiveGuard live;
  std::unique_ptr<md_server> sv(new md_server());
  sv->budget = hbm_budget_bytes;
  sv->max_runs = max_runs;
  sv->quantum = quantum_steps;
  sv->flags = flags;
  if (!(flags & MD_SERVER_FAKE_EXECUTOR)) {
    int rc = device_ready();
    if (rc) return rc;
    HIPCHK(hipGetDevice(&sv->device));
    HIPCHK(hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking));
  }
  md_server* p = sv.release();
  live.keep = true;
  p->th = std::thread(server_loop, p);
  *out = p;
  return MD_OK;
}

extern "C" int md_server_create(size_t hbm_budget_bytes, int max_runs, md_server** out) {
  return md_server_create_ex(hbm_budget_bytes, max_runs, 0, 0, out);
}

extern "C" int md_submit(md_server* sv, const md_run_desc* run, uint64_t* ticket) {
  if (!sv || !run || !ticket) return fail(MD_EINVAL, "bad arguments");
  DGeom g;
  int rc = make_geom(run->box, run->slices, run->rc, run->dt, run->precision, &g);
  if (rc) return rc;
  if (run->n < 0 || (run->n > 0 && (!run->pos || !run->vel)) || run->steps < 0 || run->energy_every < 0)
    return fail(MD_EINVAL, "bad run arrays or step counts");
  if ((rc = check_positions(g, run->n, run->pos, run->vel))) return rc;
  auto r = std::make_shared<ServedRun>();
  r->d = *run;
  r->d.pos = r->d.vel = nullptr;
  r->fp = served_footprint(g, run->n, sv->quantum);
  if (r->fp > (int64_t)sv->budget)
    return fail(MD_ENOMEM, "run needs %lld device bytes, budget is %zu", (long long)r->fp, sv->budget);
  r->pos.assign(run->pos, run->pos + 3 * run->n);
  r->vel.assign(run->vel, run->vel + 3 * run->n);
  r->res.tag = run->tag;
  std::lock_guard<std::mutex> lk(sv->mu);
  if ((int64_t)sv->queue.size() >= MD_SERVER_MAX_QUEUED)
    return fail(MD_EBUSY, "%d runs already wait for admission", MD_SERVER_MAX_QUEUED);
  r->ticket = sv->next_ticket++;
  r->res.t_submit = sv->now();
  sv->runs[r->ticket] = r;
  sv->queue.push_back(r);
  *ticket = r->ticket;
  sv->cv.notify_all();
  return MD_OK;
}

extern "C" int md_poll(md_server* sv, uint64_t ticket, md_result* out) {
  if (!sv) return fail(MD_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->runs.find(ticket);
  if (it == sv->runs.end()) return fail(MD_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  ServedRun& r = *it->second;
  if (r.status == MD_PENDING) return MD_PENDING;
  if (out) *out = r.res;
  const int st = r.status;
  r.polled = true;
  if (!r.d.keep_state || st != MD_OK) sv->runs.erase(it);
  return st;
}

extern "C" int md_fetch_state(md_server* sv, uint64_t ticket, double* pos, double* vel) {
  if (!sv) return fail(MD_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->runs.find(ticket);
  if (it == sv->runs.end()) return fail(MD_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  ServedRun& r = *it->second;
  if (r.status == MD_PENDING) return MD_PENDING;
  if (r.status != MD_OK) return fail(r.status, "run failed");
  if (!r.d.keep_state) return fail(MD_ESTATE, "run was not submitted with keep_state");
  const size_t m = (size_t)3 * r.d.n;
  if (pos && m) std::memcpy(pos, r.out_pos.data(), m * sizeof(double));
  if (vel && m) std::memcpy(vel, r.out_vel.data(), m * sizeof(double));
  sv->runs.erase(it);
  return MD_OK;
}

extern "C" int md_server_stats(md_server* sv, int64_t* queued, int64_t* running, int64_t* done,
                               int64_t* bytes_in_use, int64_t* launches) {
  if (!sv) return fail(MD_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (queued) *queued = (int64_t)sv->queue.size();
  if (running) *running = (int64_t)sv->running.size();
  if (done) *done = sv->ndone;
  if (bytes_in_use) *bytes_in_use = sv->in_use;
  if (launches) *launches = sv->launches;
  return MD_OK;
}

extern "C" int md_server_times(md_server* sv, double* admit_s, double* launch_s, double* finish_s,
                               double* idle_s) {
  if (!sv) return fail(MD_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (admit_s) *admit_s = sv->t_admit;
  if (launch_s) *launch_s = sv->t_launch;
  if (finish_s) *finish_s = sv->t_finish;
  if (idle_s) *idle_s = sv->t_idle;
  return MD_OK;
}

extern "C" int md_server_destroy(md_server* sv) {
  if (!sv) return fail(MD_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->th.joinable()) sv->th.join();
  for (auto& r : sv->running)
    if (r->sim) md_free(r->sim);
  sv->running.clear();
  sv->queue.clear();
  sv->runs.clear();
  sv->ls.release();
  if (sv->stream) (void)hipStreamDestroy(sv->stream);
  delete sv;
  g_live--;
  return MD_OK;
}
