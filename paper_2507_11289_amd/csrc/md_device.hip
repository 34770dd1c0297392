// md_device.hip -- gfx950 kernels of the slice-streaming Lennard-Jones path.
//
// Paper: "Cyclic Data Streaming on GPUs for Short Range Stencils Applied to
// Molecular Dynamics" (arXiv 2507.11289).
//   * Sec. 4: truncated-and-shifted LJ 12-6 (sigma = epsilon = 1), cells of edge > rc,
//     neighbours in the own and adjacent cells, input/output order 1 in x.
//   * Algorithm 1: pair force F_abs = 24 (2 r^-12 - r^-6) / r^2 on r_ij for
//     r_ij . r_ij <= rc^2, energy and virial accumulation, velocity-Verlet update.
//   * Sec. 4.1: molecules processed in cell order so that neighbouring lanes share
//     neighbour lists (md_fill_mol_work_list / md_v3a); new velocities (md_v3aa);
//     energy/virial collection (stat_collect); new positions and the runtime decision
//     in which slice a molecule is stored (md_v3b).
//   * Sec. 3.1-3.3 / Table 1: a slice is processed once its neighbours are present; on
//     one GPU this becomes a persistent kernel whose work items follow per-slice
//     counters (slice i advances t -> t+1 once i-1 and i+1 reached t).
//
// One wavefront owns one cell at a time.  A cell's atoms sit in slots 0..n-1 of its
// 64-slot block, ordered by id, so every atom's force sum has a fixed order and the
// trajectory is bitwise independent of the order in which work items run.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "md_internal.h"

namespace mdk {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Device-memory pointers in the global address space.  The buffers reach the kernels
// as generic pointers (inside the run arguments), which would make every access a flat
// one: flat accesses count against the LDS counter as well, so each LDS wait would also
// wait for all outstanding cell loads and stores.
#define GLOBAL __attribute__((address_space(1)))
typedef GLOBAL double gdouble;
typedef GLOBAL uint32_t guint32;
template <class T> __device__ __forceinline__ GLOBAL T* gptr(T* p) { return (GLOBAL T*)p; }
template <class T> __device__ __forceinline__ const GLOBAL T* gptr(const T* p) { return (const GLOBAL T*)p; }

__device__ __forceinline__ gdouble* cblk(unsigned char* base, int c) {
  return (gdouble*)(base + (size_t)c * CELL_BYTES);
}
__device__ __forceinline__ const gdouble* cblk(const unsigned char* base, int c) {
  return (const gdouble*)(base + (size_t)c * CELL_BYTES);
}
__device__ __forceinline__ guint32* cids(gdouble* b) {
  return (guint32*)(b + CELL_DOUBLES);
}
__device__ __forceinline__ const guint32* cids(const gdouble* b) {
  return (const guint32*)(b + CELL_DOUBLES);
}
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef float vf3 __attribute__((ext_vector_type(3)));
struct dpos {
  double x, y, z;
};
typedef GLOBAL vf4 gvf4;
// FP32 corner-relative positions (x, y, z, 0) of the slots
__device__ __forceinline__ gvf4* crel(gdouble* b) { return (gvf4*)(cids(b) + CELL_CAP); }
__device__ __forceinline__ const gvf4* crel(const gdouble* b) { return (const gvf4*)(cids(b) + CELL_CAP); }

// FP64 sums, differences and products rounded one operation at a time, in the order
// written, as the oracle computes them.  They are never fused into multiply-adds: this
// toolchain's __dadd_rn / __dmul_rn are plain operators, and the default contraction
// mode fuses a product feeding a sum into one FMA (one rounding instead of two), which
// would move r^2 off the oracle's value and could flip a cutoff decision.
__device__ __forceinline__ double add_rn(double a, double b) {
#pragma clang fp contract(off)
  return a + b;
}
__device__ __forceinline__ double sub_rn(double a, double b) {
#pragma clang fp contract(off)
  return a - b;
}
__device__ __forceinline__ double mul_rn(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}

__device__ __forceinline__ unsigned ld_relaxed(const uint32_t* p) {
  return __hip_atomic_load(gptr(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// XCD (L2 domain) running the calling wave: bits [3:0] of the XCC_ID hardware register.
__device__ __forceinline__ int xcc_id() {
  return (int)(__builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & 0xFu);
}

// Work queue of slice s of a run: queue x holds the slices [xfirst[x], xfirst[x + 1]).
__device__ __forceinline__ int slice_queue(const RunArgs& ra, int nq, int s) {
  int x = 0;
  for (int q = 1; q < nq; q++) x += s >= ra.xfirst[q] ? 1 : 0;
  return x;
}

__device__ __forceinline__ void raise_error(uint32_t* err, uint32_t* abort_flag, uint32_t bits) {
  __hip_atomic_fetch_or(err, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (abort_flag) __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cell coordinate along one axis: floor(x * (1/l)) with one IEEE multiply, clamped
// to [0, G-1] (a coordinate equal to L after wrapping belongs to the last cell; NaN
// gives 0).  Branch-free.
__device__ __forceinline__ int coord_cell(double x, double inv_l, int G) {
  const double f = floor(mul_rn(x, inv_l));
  return (int)fmin(fmax(f, 0.0), (double)(G - 1));
}

// Position x relative to the corner gc l of its cell, rounded once to FP32 (stored beside
// the FP64 position for the FP32 pair path).
__device__ __forceinline__ float corner_rel(double x, int gc, double l) {
  return (float)sub_rn(x, mul_rn((double)gc, l));
}

// n / d for 0 <= n < 2^51 from inv = 1/d rounded to FP64: the quotient (n + 1/2) / d lies
// at least 1/(2d) from an integer, and its FP64 product with inv is within
// (n + 1/2) 2^-52 / d < 1/(2d) of it, so truncation gives the integer quotient (a few
// FP64 operations instead of an integer division sequence).
__device__ __forceinline__ int qdiv(int n, double inv) {
  return (int)mul_rn(add_rn((double)n, 0.5), inv);
}

__device__ __forceinline__ int global_cell(const DGeom& g, int gx, int gy, int gz) {
  const int s = qdiv(gx, g.inv_ncx);
  return s * g.cps + ((gx - s * g.ncx) * g.G[1] + gy) * g.G[2] + gz;
}

__device__ __forceinline__ void cell_xyz(const DGeom& g, int c, int& gx, int& gy, int& gz) {
  const int s = qdiv(c, g.inv_cps);
  const int local = c - s * g.cps;
  const int t = qdiv(local, g.inv_G[2]);
  gz = local - t * g.G[2];
  const int u = qdiv(t, g.inv_G[1]);
  gy = t - u * g.G[1];
  gx = s * g.ncx + u;
}

// Minimum image of one component (the box is at least 3 cells, so the image within
// rc is unique).
__device__ __forceinline__ double min_img(double d, double L, double h) {
  return d > h ? sub_rn(d, L) : (d < -h ? add_rn(d, L) : d);
}

__device__ __forceinline__ double r2_exact(double dx, double dy, double dz) {
  return add_rn(add_rn(mul_rn(dx, dx), mul_rn(dy, dy)), mul_rn(dz, dz));
}

// Branch-free: both candidates are formed and one is selected.
__device__ __forceinline__ double wrap1(double x, double L) {
  const double below = sub_rn(x, L), above = add_rn(x, L);
  return x >= L ? below : (x < 0.0 ? above : x);
}

// 1/x in FP64 from the hardware reciprocal and two Newton steps (within one ulp).
__device__ __forceinline__ double recip64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// ---------------------------------------------------------------------------
// Block staging.  A workgroup works on up to BZ consecutive cells of one z-column
// (one cell per wave).  Their 27-cell neighbourhoods form a 3 x 3 x (nb + 2) block of
// cells, staged once in LDS in layer-major order (z layer, then dx, then dy), so the
// 27 neighbours of the cell of wave w are the contiguous entries of layers w .. w+2.
// ---------------------------------------------------------------------------
constexpr int BZ = BLOCK_CELLS;         // cells per block, one per wave
constexpr int BLAYERS = BZ + 2;         // staged z layers
constexpr int BCELLS = 9 * BLAYERS;     // staged cells
constexpr int CAPB = 27 * CELL_CAP;     // staged atoms at most (one full neighbourhood)
constexpr int QPAD = 16;                // far sentinels after the staged atoms (FP32)
constexpr float FAR_Q = 1e15f;          // sentinel coordinate: far from everything, |q|^2 finite

// FP32 far sentinel entry, built where it is stored: a copy kept across the block loop
// does not fit the register budget and was spilled to scratch memory, costing a reload
// and a wait for all outstanding memory operations in every staging
__device__ __forceinline__ float4 far_entry() {
  float c = FAR_Q, n = 3.0f * FAR_Q * FAR_Q;
  asm volatile("" : "+v"(c), "+v"(n));
  return make_float4(c, c, c, n);
}

struct BlockHdr {
  int nb_cell[BCELLS];     // global cell of staged cell m
  int cnt[BCELLS];         // atoms of staged cell m
  int pre[BCELLS + 1];     // first staged entry of cell m
  double org[3];           // origin of the block's FP32 coordinates
  int gx, gy, z0;          // the block: cells z0 .. z0 + nb - 1 of column (gx, gy)
  int nb;                  // cells of this block (after the capacity check)
  int nst;                 // staged cells, 9 (nb + 2)
  int wrap;                // some staged cell is a periodic image
  int wrap_col;            // the column touches a periodic boundary in x or y
  int wrap_layer[BLAYERS]; // z layer is a periodic image
};

template <int PREC> struct BlockLDS;
constexpr int GMASKS = 4;  // pre-filter mask words kept per lane: one group of the pair walk and the
                           // guard-band pass (32 tiles)
template <> struct BlockLDS<1> {  // FP32: positions relative to the block origin, |q|^2
  BlockHdr hb[2];                 // headers of the current and the next block
  float4 qoff[2][BCELLS];         // per header: corner of staged cell m relative to the block
                                  // origin, (k l) rounded to FP32 per axis
  float4 q[CAPB + QPAD];
  unsigned gmask[WAVES][GMASKS + 1][64];  // each wave's pass-1 marks of its current atom batch
                                         // (and a padding word read ahead, never used)
};
template <> struct BlockLDS<0> {  // FP64: raw positions, plus per entry the periodic image
  BlockHdr hb[2];                 // and the FP32 |q|^2 of the matrix-core pre-filter; headers
                                  // of the current and the next block
  double x[CAPB + QPAD], y[CAPB + QPAD], z[CAPB + QPAD];
  float qn[CAPB + QPAD];
  uint8_t img[CAPB + QPAD];       // (sx + 1) | (sy + 1) << 2 | (sz + 1) << 4: image shift s L
};

// Image code of a staged entry without a periodic shift.
constexpr uint8_t IMG_NONE = 1 | (1 << 2) | (1 << 4);

struct ForceOut {
  double fx, fy, fz;  // force on the lane's atom (lanes < n)
  double x[3], v[3];  // FP64 position and stored velocity of the lane's atom
  uint32_t id;        // its id
  double uh, wh;      // half sums of pair energy / pair virial
  unsigned pc;        // in-range partners (count mode)
  int n;              // atoms in the cell (uniform per wave)
  int total;          // candidates in the 27 cells, self included (uniform per wave)
  int c;              // global cell of the wave (-1: no cell in this block)
};

// Partial sums of one i-atom held by one lane.
template <class R> struct Acc {
  R fx, fy, fz;
  double u, w;
  unsigned pc;
};

template <class R> __device__ __forceinline__ void acc_init(Acc<R>& a) {
  a.fx = a.fy = a.fz = (R)0;
  a.u = a.w = 0.0;
  a.pc = 0;
}

// LJ pair-force factor F_abs = 24 (2 r^-12 - r^-6) / r^2 = ir2 ir6 (48 ir6 - 24).
template <class R> __device__ __forceinline__ R force_factor(R ir2, R ir6) {
  return (ir6 * (ir6 * (R)48 - (R)24)) * ir2;
}

// FP32 pair term of a pre-filtered pair (Algorithm 1 loop body): the range decision and
// arithmetic of a pair-by-pair FP32 loop.  Returns rb - lo_bits (unsigned, rb = bits of
// r2 minus 1): below hi_bits - lo_bits exactly for a guard-band pair, which is then
// decided again in FP64; pairs in range, out of range and the self pair give more.
template <bool ENERGY, bool COUNT>
__device__ __forceinline__ unsigned pair32_in(const float4& qi, const float4& q, unsigned lo_bits, float ucf,
                                              Acc<float>& a) {
  const float dx = qi.x - q.x, dy = qi.y - q.y, dz = qi.z - q.z;
  const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  // u = rb - lo_bits (mod 2^32) in one subtraction; rb < lo_bits (in range) exactly when
  // u > ~lo_bits, which r2 = 0 (u = ~lo_bits) is not
  const unsigned u = __float_as_uint(r2) - (lo_bits + 1u);
  const bool in = u > ~lo_bits;
  const float ir2 = __builtin_amdgcn_rcpf(r2);
  const float ir6 = ir2 * ir2 * ir2;
  float fr = force_factor(ir2, ir6);
  fr = in ? fr : 0.0f;
  a.fx = fmaf(fr, dx, a.fx);
  a.fy = fmaf(fr, dy, a.fy);
  a.fz = fmaf(fr, dz, a.fz);
  if (ENERGY) {
    a.u += in ? (double)(4.0f * ir6 * (ir6 - 1.0f) - ucf) : 0.0;
    a.w += in ? (double)(24.0f * ir6 * fmaf(2.0f, ir6, -1.0f)) : 0.0;
  }
  if (COUNT) a.pc += in ? 1u : 0u;
  return u;
}

// The same FP32 pair term, added unconditionally (guard-band pairs found in range).
template <bool ENERGY, bool COUNT>
__device__ __forceinline__ void pair32_add(float dx, float dy, float dz, float r2, float ucf, Acc<float>& a) {
  const float ir2 = __builtin_amdgcn_rcpf(r2);
  const float ir6 = ir2 * ir2 * ir2;
  const float fr = force_factor(ir2, ir6);
  a.fx = fmaf(fr, dx, a.fx);
  a.fy = fmaf(fr, dy, a.fy);
  a.fz = fmaf(fr, dz, a.fz);
  if (ENERGY) {
    a.u += (double)(4.0f * ir6 * (ir6 - 1.0f) - ucf);
    a.w += (double)(24.0f * ir6 * fmaf(2.0f, ir6, -1.0f));
  }
  if (COUNT) a.pc += 1u;
}

// FP64 pair; WRAP applies the minimum-image rule to every component.
template <bool ENERGY, bool COUNT, bool WRAP>
__device__ __forceinline__ void pair64(const DGeom& g, double xi, double yi, double zi, double xj, double yj,
                                       double zj, Acc<double>& a) {
  double dx = sub_rn(xi, xj), dy = sub_rn(yi, yj), dz = sub_rn(zi, zj);
  if (WRAP) {
    dx = min_img(dx, g.L[0], g.halfL[0]);
    dy = min_img(dy, g.L[1], g.halfL[1]);
    dz = min_img(dz, g.L[2], g.halfL[2]);
  }
  const double r2 = r2_exact(dx, dy, dz);
  const bool in = (r2 <= g.rc2) & (r2 > 0.0);
  const double ir2 = recip64(r2);
  const double ir6 = ir2 * ir2 * ir2;
  double fr = force_factor(ir2, ir6);
  fr = in ? fr : 0.0;
  a.fx = fma(fr, dx, a.fx);
  a.fy = fma(fr, dy, a.fy);
  a.fz = fma(fr, dz, a.fz);
  if (ENERGY) {
    a.u += in ? 4.0 * ir6 * (ir6 - 1.0) - g.uc : 0.0;
    a.w += in ? 24.0 * ir6 * fma(2.0, ir6, -1.0) : 0.0;
  }
  if (COUNT) a.pc += in ? 1u : 0u;
}

// Staging of the block of the column (gx, gy) whose cells start at z0 (at most nb_max
// of them, all in the column).  One wave prepares each block's header:
//   hdr_issue: lane m loads the atom count of staged cell m -- one block ahead, so the
//     counts arrive while the previous block is integrated;
//   hdr_commit: prefix of the counts, capacity check, header (double-buffered, so the
//     next block's header is written while the current one is in use).
// Then the staging waves (all four, or the three that are not finishing the previous
// block) stage the block (stage_entries): each quarter wave (16 lanes) takes whole staged
// cells, one atom slot per lane: cell NQ i + 4 s + quarter of staging wave s for i < SR
// (NQ = 4 x staging waves), all of them loaded at once (one memory round trip for the
// whole block), then written into LDS at the cell's place in the compact staged list.
// The slots past the 16th of a quarter's cells follow, concatenated, in one more batch.
// ---------------------------------------------------------------------------
template <int NSW> struct StageShape {
  static constexpr int NQ = 4 * NSW;                 // quarter waves staging
  static constexpr int SR = (BCELLS + NQ - 1) / NQ;  // staged cells per quarter wave
  static_assert(NQ * SR <= 64, "a staged cell index must name a lane of the wave");
};

// threadIdx.x behind an empty asm: index arithmetic derived from it stays where it is
// used instead of being hoisted out of the block loop and held in registers through the
// pair loop.
__device__ __forceinline__ int opaque_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

struct StageRegs {
  int gx, gy, z0, nb_max;
  int nc, cnt;  // lane m < 9 (nb_max + 2): global cell and atom count of staged cell m
};

__device__ __forceinline__ void staged_cell_xyz(int gx, int gy, int z0, int m, int& nx, int& ny, int& nz) {
  const int lay = m / 9, r = m % 9;
  nx = gx + r / 3 - 1;
  ny = gy + r % 3 - 1;
  nz = z0 - 1 + lay;
}

__device__ __forceinline__ void hdr_issue(const DGeom& g, const uint32_t* ncnt, int gx, int gy, int z0,
                                          int nb_max, StageRegs& R) {
  const int lane = __lane_id();
  R.gx = gx;
  R.gy = gy;
  R.z0 = z0;
  R.nb_max = nb_max;
  const int ncs = 9 * (nb_max + 2);
  int nc = 0;
  if (lane < ncs) {
    int nx, ny, nz;
    staged_cell_xyz(gx, gy, z0, lane, nx, ny, nz);
    nx += nx < 0 ? g.G[0] : (nx >= g.G[0] ? -g.G[0] : 0);
    ny += ny < 0 ? g.G[1] : (ny >= g.G[1] ? -g.G[1] : 0);
    nz += nz < 0 ? g.G[2] : (nz >= g.G[2] ? -g.G[2] : 0);
    nc = global_cell(g, nx, ny, nz);
  }
  R.nc = nc;
  R.cnt = lane < ncs ? (int)gptr(ncnt)[nc] : 0;
}

// wrap: some staged cell of the block is a periodic image (its coordinates are shifted
// by a box length); without it the shift is 0 and x + 0 = x exactly.
// FP32 origin of a block: the column corner at the start of z0's aligned group of BZ
// cells, so a pair's FP32 arithmetic depends on the cell only, not on how cells form
// blocks.
__device__ __forceinline__ void block_origin(const DGeom& g, int gx, int gy, int z0, double o[3]) {
  o[0] = mul_rn((double)gx, g.l[0]);
  o[1] = mul_rn((double)gy, g.l[1]);
  o[2] = mul_rn((double)(z0 - z0 % BZ), g.l[2]);
}

// FP32 coordinate of a staged position: (x + s L) - o, rounded once to FP32.
__device__ __forceinline__ float rel32(double x, int s, double L, double o) {
  return (float)sub_rn(add_rn(x, (double)s * L), o);
}

// wrap: some staged cell of the block is a periodic image (its coordinates are shifted
// by a box length); without it every shift is 0.
// FP32: the staged coordinate is the atom's corner-relative FP32 position plus its staged
// cell's corner relative to the block origin (qoff), one FP32 addition per axis.  The cell
// indices of the corner are taken unwrapped, so a periodic image needs no shift.
// FP64: raw positions for the exact FP64 pair terms, plus the image code and the FP32 |q|^2
// the pre-filter rebuilds its FP32 coordinates from (x + s L) - o, rounded once.
__device__ __forceinline__ void stage_put(const DGeom& g, const BlockHdr& H, BlockLDS<1>& L, const float4& off,
                                          int m, int p, float rx, float ry, float rz) {
  const float qx = rx + off.x, qy = ry + off.y, qz = rz + off.z;
  // w: |q|^2, the norm term of the matrix-core distance test
  L.q[p] = make_float4(qx, qy, qz, fmaf(qx, qx, fmaf(qy, qy, qz * qz)));
}
__device__ __forceinline__ void stage_put(const DGeom& g, const BlockHdr& H, BlockLDS<0>& L, const double o[3],
                                          int m, int p, double x, double y, double z, bool wrap) {
  int sx = 0, sy = 0, sz = 0;
  if (wrap) {
    int nx, ny, nz;
    staged_cell_xyz(H.gx, H.gy, H.z0, m, nx, ny, nz);
    sx = nx < 0 ? -1 : (nx >= g.G[0] ? 1 : 0);
    sy = ny < 0 ? -1 : (ny >= g.G[1] ? 1 : 0);
    sz = nz < 0 ? -1 : (nz >= g.G[2] ? 1 : 0);
  }
  const float qx = rel32(x, sx, g.L[0], o[0]), qy = rel32(y, sy, g.L[1], o[1]), qz = rel32(z, sz, g.L[2], o[2]);
  L.x[p] = x;
  L.y[p] = y;
  L.z[p] = z;
  L.qn[p] = fmaf(qx, qx, fmaf(qy, qy, qz * qz));
  L.img[p] = (uint8_t)((sx + 1) | ((sy + 1) << 2) | ((sz + 1) << 4));
}

// Header of the block from the counts of hdr_issue: prefix, capacity check (the largest
// nb whose 9 (nb + 2) cells fit; nb = 1 always fits).  One wave.
template <int PREC>
__device__ void hdr_commit(const DGeom& g, const StageRegs& R, BlockLDS<PREC>& L, int hbi) {
  BlockHdr& H = L.hb[hbi];
  const int lane = __lane_id();
  int incl = R.cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  int nb = R.nb_max;
  while (nb > 1 && __shfl(incl, 9 * (nb + 2) - 1) > CAPB) nb--;
  if (lane < BCELLS) {
    H.nb_cell[lane] = R.nc;
    H.cnt[lane] = R.cnt;
    H.pre[lane] = incl - R.cnt;
  }
  if (lane == BCELLS - 1) H.pre[BCELLS] = incl;
  if (lane == 0) {
    H.gx = R.gx;
    H.gy = R.gy;
    H.z0 = R.z0;
    H.nb = nb;
    H.nst = 9 * (nb + 2);
    H.wrap_col = R.gx == 0 || R.gx == g.G[0] - 1 || R.gy == 0 || R.gy == g.G[1] - 1;
    H.wrap = H.wrap_col || R.z0 == 0 || R.z0 + nb >= g.G[2];
    if constexpr (PREC == 0) block_origin(g, R.gx, R.gy, R.z0, H.org);
  }
  if (lane < BLAYERS) {
    const int nz = R.z0 - 1 + lane;
    H.wrap_layer[lane] = nz < 0 || nz >= g.G[2];
  }
  if constexpr (PREC == 1) {
    if (lane < BCELLS) {
      // staged cell lane: x, y offsets -1..1 from the column, z from the aligned group start
      // (the lane index is recomputed so that its conversions are not held across the block
      // loop)
      const int ln = opaque_tid() & 63;
      const int r = ln % 9;
      const int kx = r / 3 - 1, ky = r % 3 - 1, kz = ln / 9 - 1 + R.z0 % BZ;
      L.qoff[hbi][ln] = make_float4((float)mul_rn((double)kx, g.l[0]), (float)mul_rn((double)ky, g.l[1]),
                                    (float)mul_rn((double)kz, g.l[2]), 0.0f);
    }
  }
}

// Atoms of the block's own cells, in cell order (at most BZ cells).
__device__ __forceinline__ int block_atoms(const BlockHdr& H) {
  int t = 0;
#pragma unroll
  for (int q = 0; q < BZ; q++) t += q < H.nb ? H.cnt[9 * (q + 1) + 4] : 0;
  return t;
}

// Stage the block of header hbi into LDS with NSW waves; the calling wave is staging wave
// sw (0 .. NSW - 1).  The LDS entries must be free and the header complete on entry; no
// barrier.
template <int PREC, int NSW>
__device__ void stage_entries(const DGeom& g, const unsigned char* cells, int hbi, BlockLDS<PREC>& L, int sw) {
  constexpr int NQ = StageShape<NSW>::NQ, SR = StageShape<NSW>::SR;
  const BlockHdr& H = L.hb[hbi];
  // the staged position of a slot: FP32 corner-relative (FP32 pair path: x, y, z in one
  // 12-byte load kept whole, so no register of it is reused, and nothing waits for the load,
  // before the position is used) or FP64
  typedef typename std::conditional<PREC == 1, vf3, dpos>::type PT;
  auto load_pos = [&](const gdouble* jb, int k, PT& r) {
    if constexpr (PREC == 1) {
      r = *reinterpret_cast<const GLOBAL vf3*>(crel(jb) + k);
    } else {
      r.x = jb[k];
      r.y = jb[CELL_CAP + k];
      r.z = jb[2 * CELL_CAP + k];
    }
  };
  const int lane = __lane_id();
  const int nst = H.nst;
  const bool wrap = H.wrap;
  if (sw == 0 && lane < QPAD) {
    // far sentinels after the last staged atom: a pair-loop read past the end of the
    // list finds no partner in range
    const int stot = H.pre[nst];
    if constexpr (PREC == 1) {
      L.q[stot + lane] = far_entry();
    } else {
      L.x[stot + lane] = L.y[stot + lane] = L.z[stot + lane] = (double)FAR_Q;
      L.qn[stot + lane] = 3.0f * FAR_Q * FAR_Q;
      L.img[stot + lane] = IMG_NONE;
    }
  }
  // staged cell of round 0 (round i: m0 + NQ i), i.e. 4 sw + quarter; recomputed here so
  // that the per-round indices are not hoisted out of the block loop and held in registers
  const int st = NSW == WAVES ? opaque_tid() : ((sw << 6) | (opaque_tid() & 63));
  const int m0 = st >> 4, j = st & 15;
  int pi[SR];  // staged entry of the lane's slot, or -1
  int ex[SR];  // the cell's atoms past its 16th (0 if none, or if not staged)
  PT r[SR];
  // raised wave priority while the loads are found and issued: the SIMD's other waves are
  // mostly in VALU-heavy pair loops, and an early issue lets the memory round trip overlap
  // their work
  __builtin_amdgcn_s_setprio(2);
#pragma unroll
  for (int i = 0; i < SR; i++) {
    const int m = m0 + NQ * i;
    const int ms = m < BCELLS ? m : 0;
    const int cnt = m < nst ? H.cnt[ms] : 0;
    const int cell = H.nb_cell[ms];
    const bool have = j < cnt;
    pi[i] = have ? H.pre[ms] + j : -1;
    ex[i] = max(cnt - 16, 0);
    r[i] = PT{0, 0, 0};
    if (have) load_pos(cblk(cells, cell), j, r[i]);
  }
  // the slots past the 16th of the quarter's cells, concatenated: 16 of them per pass, the
  // first pass issued with the loads above; ec[i] = extra slots of the rounds before i
  int ec[SR + 1];
  ec[0] = 0;
#pragma unroll
  for (int i = 0; i < SR; i++) ec[i + 1] = ec[i] + ex[i];
  const int etot = ec[SR];
  auto extra = [&](int v, int& m, int& p, PT& rv) {
    int i = 0, base = 0;
#pragma unroll
    for (int t = 1; t < SR; t++)
      if (v >= ec[t]) {
        i = t;
        base = ec[t];
      }
    const int k = 16 + v - base;
    m = m0 + NQ * i;
    p = -1;
    rv = PT{0, 0, 0};
    if (v < etot) {
      p = H.pre[m] + k;
      load_pos(cblk(cells, H.nb_cell[m]), k, rv);
    }
  };
  int me, pe;
  PT re;
  extra(j, me, pe, re);
  __builtin_amdgcn_s_setprio(0);
  double o[3];
  if constexpr (PREC == 0) block_origin(g, H.gx, H.gy, H.z0, o);
  auto put = [&](int m, int p, const PT& rv) {
    if constexpr (PREC == 1)
      stage_put(g, H, L, L.qoff[hbi][m], m, p, rv.x, rv.y, rv.z);
    else
      stage_put(g, H, L, o, m, p, rv.x, rv.y, rv.z, wrap);
  };
#pragma unroll
  for (int i = 0; i < SR; i++)
    if (pi[i] >= 0) put(m0 + NQ * i, pi[i], r[i]);
  if (pe >= 0) put(me, pe, re);
  // every round's registers are read on every path: otherwise a load whose value is (in
  // the compiler's view) left unread looks outstanding later, and a later wait for other
  // loads also waits for it
#pragma unroll
  for (int i = 0; i < SR; i++) asm volatile("" ::"v"(r[i].x), "v"(r[i].y), "v"(r[i].z));
  asm volatile("" ::"v"(re.x), "v"(re.y), "v"(re.z));
  // more than 16 extra slots in some quarter (dense cells): the rest, a pass at a time
  for (int v0 = 16; __ballot(v0 < etot); v0 += 16) {
    extra(v0 + j, me, pe, re);
    if (pe >= 0) put(me, pe, re);
    // read on every path: a load left in flight here would make a later write of these
    // registers wait for the memory counter (and with it for every later load)
    asm volatile("" ::"v"(re.x), "v"(re.y), "v"(re.z));
  }
}

// Position, velocity and id of own atoms of the block of header H into own.  own_mode 1:
// every wave loads those of its own cell (none if the capacity check dropped it); 2: wave
// tw loads those of all the block's cells, atom l of them (in cell order) on lane l (at
// most 64).  The pair loops wait for no memory operation, so the loads arrive during them.
__device__ __forceinline__ void own_load(const unsigned char* cells, const BlockHdr& H, ForceOut& own, int own_mode,
                                         int tw) {
  const int lane = __lane_id();
  const int w = threadIdx.x >> 6;
  if (own_mode == 1 || (own_mode == 2 && w == tw)) {
    // own_mode 2: cell q of the block holds atoms [P_q, P_q + n_q) of the lanes
    int q = w, k = lane, nq = w < H.nb ? H.cnt[9 * (w + 1) + 4] : 0;
    if (own_mode == 2) {
      int nr[BZ], P[BZ + 1];
      P[0] = 0;
#pragma unroll
      for (int r = 0; r < BZ; r++) {
        nr[r] = r < H.nb ? H.cnt[9 * (r + 1) + 4] : 0;
        P[r + 1] = P[r] + nr[r];
      }
      q = (lane >= P[1] ? 1 : 0) + (lane >= P[2] ? 1 : 0) + (lane >= P[3] ? 1 : 0);
      k = lane - (q == 0 ? 0 : (q == 1 ? P[1] : (q == 2 ? P[2] : P[3])));
      nq = q == 0 ? nr[0] : (q == 1 ? nr[1] : (q == 2 ? nr[2] : nr[3]));
    }
    if (k < nq) {
      const gdouble* ib = cblk(cells, H.nb_cell[9 * (q + 1) + 4]);
#pragma unroll
      for (int d = 0; d < 3; d++) {
        own.x[d] = ib[d * CELL_CAP + k];
        own.v[d] = ib[(3 + d) * CELL_CAP + k];
      }
      own.id = cids(ib)[k];
    }
  }
}

// Stage the block of header hbi into LDS with all waves, then (own_mode 1 or 2) the own
// atoms' loads of own_load, issued last, once the staged entries are written.  Whole
// workgroup; the LDS entries must be free and the header complete on entry; ends with a
// barrier.
template <int PREC>
__device__ void stage_fill(const DGeom& g, const unsigned char* cells, int hbi, BlockLDS<PREC>& L, ForceOut& own,
                           int own_mode, int tw) {
  stage_entries<PREC, WAVES>(g, cells, hbi, L, threadIdx.x >> 6);
  own_load(cells, L.hb[hbi], own, own_mode, tw);
  __syncthreads();
}

typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// FP32 pair forces of every atom of the cell of wave w in the staged block (Algorithm 1,
// first loop; kernel md_v3a).  The lanes form 16 atom columns by 4 quarters: in batch u,
// lane l holds own atom a = 16 u + (l & 15) and, of every tile of 16 consecutive
// candidates of the cell's 27-cell window, the 4 candidates (l >> 4) + 4 r, r < 4 (every
// fourth one, so each lane samples the whole window).
//   Pass 1 (matrix cores): per tile, one 16x16x4 FP32 MFMA with candidate rows
//     (x, y, z, |q|^2), atom columns (-2x, -2y, -2z, 1) and accumulator |q_a|^2 - pre
//     gives r2 - pre for all 256 pairs; its error is far below the margin of pre over
//     the guard band, so the sign bits mark a superset of the pairs in range.
//   Pass 2 (vector ALU): the marked pairs two at a time in a fixed order, with the exact
//     FP32 arithmetic and range decision of a pair-by-pair loop; a running minimum of
//     rb - lo_bits tells whether any pair fell in the guard band, and those pairs are
//     then decided in FP64 (revisiting the lane's marked candidates from saved masks).
// An atom's four quarter partials are added as (q0 + q1) + (q2 + q3), so every sum has a
// fixed order.  Wave-level (no barrier).
template <bool ENERGY, bool COUNT>
__device__ void block_force32(const DGeom& g, const unsigned char* cells, const BlockHdr& H, BlockLDS<1>& L,
                              int w, ForceOut& o) {
  const int lane = __lane_id();
  const int col = lane & 15, quarter = lane >> 4;
  const int n_i = o.n;
  const int ci = 9 * (w + 1) + 4;
  const int beg = H.pre[9 * w];
  const int fe = beg + o.total;
  const int si = H.pre[ci];  // own atoms in the staged list
  // tiles of the window; the last one may reach up to 15 entries past its end, into the
  // next z layer (two cells above the own cell: out of range) or the far sentinels
  const int ntile = __builtin_amdgcn_readfirstlane((o.total + 15) >> 4);
  const unsigned lo_bits = __float_as_uint(g.rc2_lo_f), hi_bits = __float_as_uint(g.rc2_hi_f);
  const float* Lf = reinterpret_cast<const float*>(L.q);
  const char* Lb = reinterpret_cast<const char*>(L.q);
  for (int u = 0; 16 * u < n_i; u++) {
    const int a = 16 * u + col;
    const bool real = a < n_i;
    const float4 qa = real ? L.q[si + a] : make_float4(FAR_Q, FAR_Q, FAR_Q, 0.0f);
    const unsigned selfb = 16u * (unsigned)(si + a);  // own entry (only real atoms have marks)
    const float comp = quarter == 0 ? qa.x : (quarter == 1 ? qa.y : qa.z);
    // a missing atom's column is zero and its accumulator huge: never marked
    const float bop = real ? (quarter == 3 ? 1.0f : -2.0f * comp) : 0.0f;
    const float cacc = real ? qa.w - g.rc2_pre_f : 1e30f;
    const mfma_f4 cop = {cacc, cacc, cacc, cacc};
    Acc<float> A;
    acc_init(A);
    unsigned bmin = 0xffffffffu;  // least rb - lo_bits of the lane's pairs (guard band test)
    // row i = 4 r + s of a tile is candidate s + 4 r of it (lane quarter s then holds
    // every fourth candidate); the lane supplies component `quarter` of row `col`
    const float* ap = Lf + 4 * (beg + (col >> 2) + 4 * (col & 3)) + quarter;
    // one matrix op in flight per wave: the operand of each op is tied to the mask the
    // previous op completed, so the op issues only after that result has been read (and
    // no register it reads is rewritten while it runs)
    auto mark = [&](unsigned m, float av) {
      asm volatile("" : "+v"(av) : "v"(m));
      const mfma_f4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bop, cop, 0, 0, 0);
      m = __builtin_amdgcn_alignbit(m, __float_as_uint(d[0]), 31);
      m = __builtin_amdgcn_alignbit(m, __float_as_uint(d[1]), 31);
      m = __builtin_amdgcn_alignbit(m, __float_as_uint(d[2]), 31);
      return __builtin_amdgcn_alignbit(m, __float_as_uint(d[3]), 31);
    };
    for (int tg = 0; tg < ntile; tg += 8 * GMASKS) {
      // groups of up to GMASKS batches of 8 tiles; pass 1 keeps one mask word per batch
      // in LDS (the guard pass below reads them again)
      const int nw = min(GMASKS, (ntile - tg + 7) >> 3);
      for (int bi = 0; bi < nw; bi++) {
        const int tb = tg + 8 * bi;
        const int cn = min(8, ntile - tb);
        unsigned m = 0u;
        if (cn == 8) {
          // a full batch: all operand reads first, then the matrix ops
          float av[8];
#pragma unroll
          for (int t = 0; t < 8; t++) av[t] = ap[64 * (tb + t)];
#pragma unroll
          for (int t = 0; t < 8; t++) m = mark(m, av[t]);
        } else {
          for (int t = 0; t < cn; t++) m = mark(m, ap[64 * (tb + t)]);
          m <<= 32 - 4 * cn;
        }
        // after the reversal, bit b = 4 t + r marks row 4 quarter + r of tile t, i.e.
        // candidate 16 t + quarter + 4 r = 4 b + quarter of the batch
        L.gmask[w][bi][lane] = __builtin_bitreverse32(m);
      }
      // Pass 2: every lane walks its own words in order, the marked pairs two at a time
      // and lowest bit first (a fixed order), moving to its next word as soon as one is
      // used up; lanes do not wait for each other at word ends, so the wave runs for the
      // largest per-lane total rather than the sum of per-batch maxima.  A missing pair
      // is the lane's own atom (r2 = 0: neither in range nor in the band, so it adds
      // exactly nothing).  Byte offsets into the staged list.
      const unsigned fb0 = 16u * (unsigned)(beg + 16 * tg + quarter);
      const unsigned* gm = &L.gmask[w][0][lane];  // word j of the lane at gm[64 j]
      const int last = nw - 1;
      unsigned m = gm[0];
      unsigned nx = gm[64];  // the word after m (a padding word follows the last one)
      int k = 0;             // word of m
      while (m != 0u || k < last) {
        if (m == 0u) {
          m = nx;
          k++;
        }
        nx = gm[64 * (k + 1)];
        const unsigned fbb = fb0 + 2048u * (unsigned)k;
        const bool one = m != 0u;
        const unsigned b1 = (unsigned)__ffs(m) - 1u;
        m &= m - 1u;
        const bool two = m != 0u;
        const unsigned b2 = (unsigned)__ffs(m) - 1u;
        m &= m - 1u;
        const float4 q1 = *reinterpret_cast<const float4*>(Lb + (one ? fbb + 64u * b1 : selfb));
        const float4 q2 = *reinterpret_cast<const float4*>(Lb + (two ? fbb + 64u * b2 : selfb));
        const unsigned t1 = pair32_in<ENERGY, COUNT>(qa, q1, lo_bits, g.uc_f, A);
        const unsigned t2 = pair32_in<ENERGY, COUNT>(qa, q2, lo_bits, g.uc_f, A);
        bmin = min(bmin, min(t1, t2));
        // the read-ahead word is needed by the end of this iteration: its LDS read stays
        // at the top (not moved down to the next iteration's refill, which would expose
        // its latency every iteration)
        asm volatile("" ::"v"(nx));
      }
    }
    // guard band: decide those pairs in FP64 exactly as the FP64 path would.  Every pair
    // in the band was marked, so the lane visits its marked candidates again (from the
    // saved masks; a window beyond their 32 tiles is scanned in full).
    const bool flag = bmin < hi_bits - lo_bits;
    if (__ballot(flag) && flag) {
      const gdouble* iblk = cblk(cells, o.c);
      const double xi = iblk[a], yi = iblk[CELL_CAP + a], zi = iblk[2 * CELL_CAP + a];
      auto guard = [&](int f) {
        const float4 q = L.q[f];
        const float dx = qa.x - q.x, dy = qa.y - q.y, dz = qa.z - q.z;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const unsigned rb = __float_as_uint(r2) - 1u;
        if (rb >= lo_bits && rb < hi_bits) {
          // staged cell of entry f: the last one whose first entry is at or before f
          int sm = 0;
#pragma unroll
          for (int step = 32; step >= 1; step >>= 1)
            if (sm + step < BCELLS && H.pre[sm + step] <= f) sm += step;
          const gdouble* jb = cblk(cells, H.nb_cell[sm]);
          const int k = f - H.pre[sm];
          const double ex = min_img(sub_rn(xi, jb[k]), g.L[0], g.halfL[0]);
          const double ey = min_img(sub_rn(yi, jb[CELL_CAP + k]), g.L[1], g.halfL[1]);
          const double ez = min_img(sub_rn(zi, jb[2 * CELL_CAP + k]), g.L[2], g.halfL[2]);
          if (r2_exact(ex, ey, ez) <= g.rc2) pair32_add<ENERGY, COUNT>(dx, dy, dz, r2, g.uc_f, A);
        }
      };
      if (ntile <= 8 * GMASKS) {
        for (int bi = 0; 8 * bi < ntile; bi++) {
          unsigned m = L.gmask[w][bi][lane];
          const int fb = beg + 128 * bi + quarter;
          while (m) {
            const int f = fb + 4 * (__ffs(m) - 1);
            m &= m - 1u;
            if (f < fe) guard(f);
          }
        }
      } else {
        for (int t = 0; t < ntile; t++)
          for (int r = 0; r < 4; r++) {
            const int f = beg + 16 * t + quarter + 4 * r;
            if (f < fe) guard(f);
          }
      }
      // the own position is read on every path: a load of it left in flight (no band
      // pair on this lane) would make the next pair loop wait for the memory counter before
      // reusing its registers -- and that wait also covers the own-cell loads of the block,
      // which are still in flight when the first pair loop starts
      asm volatile("" ::"v"(xi), "v"(yi), "v"(zi));
    }
    // quarter partials of column col as (q0 + q1) + (q2 + q3), by two exchanges; IEEE
    // addition is commutative, so all four lanes of the column hold the same sum and lane
    // 16 u + col keeps it
    auto qsum = [](float v) {
      v += __shfl_xor(v, 16);
      return v + __shfl_xor(v, 32);
    };
    const float sx = qsum(A.fx), sy = qsum(A.fy), sz = qsum(A.fz);
    const bool keep = quarter == u && real;
    if (keep) {
      o.fx = sx;
      o.fy = sy;
      o.fz = sz;
    }
    if constexpr (ENERGY || COUNT) {
      // energy, virial and partner count (sampled steps, count mode): FP64, same order
      auto qsum64 = [](double v) {
        v += __shfl_xor(v, 16);
        return v + __shfl_xor(v, 32);
      };
      const double su = qsum64(A.u), sw = qsum64(A.w);
      unsigned sp = A.pc + __shfl_xor(A.pc, 16);
      sp += __shfl_xor(sp, 32);
      if (keep) {
        o.uh = 0.5 * su;
        o.wh = 0.5 * sw;
        o.pc = sp;
      }
    }
  }
}

// FP64 pair forces of every atom of the cell of wave w in the staged block (Algorithm 1,
// first loop; kernel md_v3a), in the lane layout and with the matrix-core pre-filter of
// the FP32 path: pass 1 rebuilds each entry's FP32 coordinates from its FP64 position,
// image code and the block origin (the values the FP32 staging would hold) and marks a
// superset of the pairs in range; pass 2 evaluates the marked pairs within the window
// with the FP64 pair arithmetic on the raw positions (minimum image where the block
// touches a periodic boundary), so every pair term and range decision is the one a
// pair-by-pair FP64 loop makes.  Quarter partials are added in quarter order.
// Wave-level (no barrier).
template <bool ENERGY, bool COUNT>
__device__ void block_force64(const DGeom& g, const BlockHdr& H, const BlockLDS<0>& L, int w, ForceOut& o) {
  const int lane = __lane_id();
  const int col = lane & 15, quarter = lane >> 4;
  const int n_i = o.n;
  const int ci = 9 * (w + 1) + 4;
  const int beg = H.pre[9 * w];
  const int fe = beg + o.total;
  const int si = H.pre[ci];  // own atoms in the staged list
  const int ntile = __builtin_amdgcn_readfirstlane((o.total + 15) >> 4);
  const bool wrap = H.wrap_col || H.wrap_layer[w] || H.wrap_layer[w + 2];
  // the component this lane supplies to the matrix ops (3: |q|^2)
  const int kc = quarter < 3 ? quarter : 2;
  const double* X = kc == 0 ? L.x : (kc == 1 ? L.y : L.z);
  const double Lk = g.L[kc], ok = H.org[kc];
  auto comp32 = [&](int f) {
    if (quarter == 3) return L.qn[f];
    const int s = (((int)L.img[f] >> (2 * kc)) & 3) - 1;
    return rel32(X[f], s, Lk, ok);
  };
  for (int u = 0; 16 * u < n_i; u++) {
    const int a = 16 * u + col;
    const bool real = a < n_i;
    const int ia = si + (real ? a : 0);
    const float qc = comp32(ia);
    const float bop = real ? (quarter == 3 ? 1.0f : -2.0f * qc) : 0.0f;
    const float cacc = real ? L.qn[ia] - g.rc2_pre_f : 1e30f;
    const mfma_f4 cop = {cacc, cacc, cacc, cacc};
    const double xi = L.x[ia], yi = L.y[ia], zi = L.z[ia];
    Acc<double> A;
    acc_init(A);
    const int r0 = beg + (col >> 2) + 4 * (col & 3);  // row col of tile 0 (as in the FP32 path)
    auto mark = [&](unsigned m, float av) {
      asm volatile("" : "+v"(av) : "v"(m));
      const mfma_f4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bop, cop, 0, 0, 0);
      m = __builtin_amdgcn_alignbit(m, __float_as_uint(d[0]), 31);
      m = __builtin_amdgcn_alignbit(m, __float_as_uint(d[1]), 31);
      m = __builtin_amdgcn_alignbit(m, __float_as_uint(d[2]), 31);
      return __builtin_amdgcn_alignbit(m, __float_as_uint(d[3]), 31);
    };
    for (int tg = 0; tg < ntile; tg += 8 * GMASKS) {
      // groups of up to GMASKS batches of 8 tiles, one mask word per batch (in registers)
      const int nw = min(GMASKS, (ntile - tg + 7) >> 3);
      unsigned wd[GMASKS];
#pragma unroll
      for (int bi = 0; bi < GMASKS; bi++) {
        wd[bi] = 0u;
        if (bi < nw) {
          const int tb = tg + 8 * bi;
          const int cn = min(8, ntile - tb);
          unsigned m = 0u;
          if (cn == 8) {
            float av[8];
#pragma unroll
            for (int t = 0; t < 8; t++) av[t] = comp32(r0 + 16 * (tb + t));
#pragma unroll
            for (int t = 0; t < 8; t++) m = mark(m, av[t]);
          } else {
            for (int t = 0; t < cn; t++) m = mark(m, comp32(r0 + 16 * (tb + t)));
            m <<= 32 - 4 * cn;
          }
          // bit b marks candidate 4 b + quarter of the batch; candidates at or past the
          // end of the window are dropped (with raw positions a periodic copy of a window
          // cell there could otherwise be counted twice)
          m = __builtin_bitreverse32(m);
          const int fb = beg + 16 * tb + quarter;
          const int nvalid = (fe - fb + 3) >> 2;
          if (nvalid < 32) m &= nvalid > 0 ? (1u << nvalid) - 1u : 0u;
          wd[bi] = m;
        }
      }
      // Pass 2: each lane walks its own words in order, the marked pairs two at a time and
      // lowest bit first, moving to its next word as soon as one is used up (lanes do not
      // wait for each other at word ends).  A missing pair is the lane's own atom (r2 = 0:
      // not in range, adds exactly nothing), so every lane makes the calls of a word-by-word
      // walk in the same order.
      const int fb0 = beg + 16 * tg + quarter;
      const int last = nw - 1;
      auto walk = [&](auto wrap_c) {
        constexpr bool WRAP = decltype(wrap_c)::value;
        // the words not yet reached move down one place at every word end (registers
        // only: an indexed choice would put them in scratch memory)
        unsigned m = wd[0], w1 = wd[1], w2 = wd[2], w3 = wd[3];
        int k = 0;
        while (m != 0u || k < last) {
          if (m == 0u) {
            k++;
            m = w1;
            w1 = w2;
            w2 = w3;
          }
          const int fbb = fb0 + 128 * k;
          const bool one = m != 0u;
          const int b1 = __ffs(m) - 1;
          m &= m - 1u;
          const bool two = m != 0u;
          const int b2 = __ffs(m) - 1;
          m &= m - 1u;
          const int f1 = one ? fbb + 4 * b1 : ia, f2 = two ? fbb + 4 * b2 : ia;
          pair64<ENERGY, COUNT, WRAP>(g, xi, yi, zi, L.x[f1], L.y[f1], L.z[f1], A);
          pair64<ENERGY, COUNT, WRAP>(g, xi, yi, zi, L.x[f2], L.y[f2], L.z[f2], A);
        }
      };
      static_assert(GMASKS == 4, "the word selection of the walk assumes four words");
      if (wrap)
        walk(std::true_type());
      else
        walk(std::false_type());
    }
    // quarter partials of column col, added in quarter order; lane 16 u + col keeps them
    const double sx = ((__shfl(A.fx, col) + __shfl(A.fx, col + 16)) + __shfl(A.fx, col + 32)) + __shfl(A.fx, col + 48);
    const double sy = ((__shfl(A.fy, col) + __shfl(A.fy, col + 16)) + __shfl(A.fy, col + 32)) + __shfl(A.fy, col + 48);
    const double sz = ((__shfl(A.fz, col) + __shfl(A.fz, col + 16)) + __shfl(A.fz, col + 32)) + __shfl(A.fz, col + 48);
    const bool keep = quarter == u && real;
    if (keep) {
      o.fx = sx;
      o.fy = sy;
      o.fz = sz;
    }
    if constexpr (ENERGY || COUNT) {
      const double su = ((__shfl(A.u, col) + __shfl(A.u, col + 16)) + __shfl(A.u, col + 32)) + __shfl(A.u, col + 48);
      const double sw = ((__shfl(A.w, col) + __shfl(A.w, col + 16)) + __shfl(A.w, col + 32)) + __shfl(A.w, col + 48);
      const unsigned sp = __shfl(A.pc, col) + __shfl(A.pc, col + 16) + __shfl(A.pc, col + 32) + __shfl(A.pc, col + 48);
      if (keep) {
        o.uh = 0.5 * su;
        o.wh = 0.5 * sw;
        o.pc = sp;
      }
    }
  }
}

// Pair forces of every atom of the cell of this wave in the staged block: header of
// the wave's cell, then the FP32 or FP64 pair loop.  Whole workgroup.
template <int PREC, bool ENERGY, bool COUNT>
__device__ void block_force(const DGeom& g, const unsigned char* cells, const BlockHdr& H, BlockLDS<PREC>& L,
                            ForceOut& o) {
  const int w = threadIdx.x >> 6;
  const bool mine = w < H.nb;
  const int ci = 9 * (w + 1) + 4;  // staged index of the wave's own cell
  o.n = mine ? H.cnt[ci] : 0;
  o.total = mine ? H.pre[9 * (w + 3)] - H.pre[9 * w] : 0;
  o.c = mine ? H.nb_cell[ci] : -1;
  o.fx = o.fy = o.fz = 0.0;
  o.uh = o.wh = 0.0;
  o.pc = 0;
  if constexpr (PREC == 1)
    block_force32<ENERGY, COUNT>(g, cells, H, L, w, o);
  else
    block_force64<ENERGY, COUNT>(g, H, L, w, o);
}

// Where the waves leave their forces for the wave that finishes the block: FP32 (the
// sums are FP32 values), in each wave's own mask words, free once its pair loop is done;
// FP64, in the staged-entry area, free once every wave's pair loop is done.  Force d of
// atom k of wave q's cell at [q * FSTRIDE + 64 d + k].
template <int PREC> struct BlockForces;
template <> struct BlockForces<1> {
  typedef float T;
  static constexpr int FSTRIDE = (GMASKS + 1) * 64;
  static constexpr bool AFTER_ALL = false;  // a wave may write as soon as its own pair loop is done
  static __device__ __forceinline__ float* at(BlockLDS<1>& L) { return reinterpret_cast<float*>(&L.gmask[0][0][0]); }
};
template <> struct BlockForces<0> {
  typedef double T;
  static constexpr int FSTRIDE = 3 * 64;
  static constexpr bool AFTER_ALL = true;   // every wave's pair loop must be done first
  static __device__ __forceinline__ double* at(BlockLDS<0>& L) { return L.x; }
};
static_assert(sizeof(unsigned) * (GMASKS + 1) * 64 >= sizeof(float) * 3 * 64, "force scratch");
static_assert(sizeof(double) * (CAPB + QPAD) >= sizeof(double) * WAVES * 3 * 64, "force scratch");

// Walk the cells [b, e) of one slice (local indices, z fastest) block by block; fn(o)
// runs on every wave after each block's forces.  Wave 0 prepares the headers: the next
// block's counts are loaded before fn and its header is written after it, while the
// other waves wait for the next block.  With OWN, the position, velocity and id of the
// wave's own atoms are loaded with the staging (in the FP32 branch below, right after
// it) and arrive during the pair loop.  With
// BTAIL, a block whose cells hold at most 64 atoms is finished by one wave (taking turns
// block by block): the waves leave their forces in LDS and fnb(H, o, forces, stride)
// runs on that wave, whose lanes hold the block's atoms in cell order; in FP32 the other
// three waves stage the next block meanwhile (see the branch below).  Whole workgroup.
template <int PREC, bool ENERGY, bool COUNT, bool OWN, bool BTAIL, class Fn, class FnB>
__device__ void for_blocks(const DGeom& g, const unsigned char* cells, const uint32_t* ncnt, int slice, int b,
                           int e, BlockLDS<PREC>& L, Fn&& fn, FnB&& fnb) {
  if (b >= e) return;
  const int w = threadIdx.x >> 6;
  // blocks stay within the column and within one aligned group of BZ cells
  auto issue = [&](int xs, StageRegs& R) {
    const int t = qdiv(xs, g.inv_G[2]);
    const int gz = xs - t * g.G[2];
    const int u = qdiv(t, g.inv_G[1]);
    const int gy = t - u * g.G[1];
    const int gx = slice * g.ncx + u;
    const int nb_max = min(min(BZ - gz % BZ, e - xs), g.G[2] - gz);
    hdr_issue(g, ncnt, gx, gy, gz, nb_max, R);
  };
  StageRegs R;
  int x = b, hb = 0, nblk = 0;
  if (w == 0) {
    issue(x, R);
    hdr_commit<PREC>(g, R, L, 0);
  }
  if constexpr (PREC == 1 && OWN && BTAIL) {
    // FP32 plain steps: the wave that finishes a block (tw, taking turns) integrates it
    // while the three others stage the next block, so the integration runs under the
    // staging's memory round trip.  The forces it reads are in the waves' mask words,
    // which the staging does not touch.  Wave 0 writes the next block's header as soon as
    // its pair loop is done, from counts loaded one block earlier (during the staging).
    typedef BlockForces<PREC> BF;
    ForceOut o;
    __syncthreads();  // the first header is complete
    if (w != WAVES - 1) stage_entries<PREC, WAVES - 1>(g, cells, 0, L, w);
    if (w == 0 && x + L.hb[0].nb < e) issue(x + L.hb[0].nb, R);
    while (true) {
      __syncthreads();  // the block is staged; the previous block is finished
      const BlockHdr& H = L.hb[hb];
      const int tw = nblk & (WAVES - 1);
      const bool one = block_atoms(H) <= 64;
      own_load(cells, H, o, one ? 2 : 1, tw);
      block_force<PREC, ENERGY, COUNT>(g, cells, H, L, o);
      // the pair loop has covered the own atoms' loads; from here on their values count
      // as plain registers, so the tail waits for no later load on their account
      asm volatile("" : "+v"(o.id), "+v"(o.x[0]), "+v"(o.x[1]), "+v"(o.x[2]), "+v"(o.v[0]), "+v"(o.v[1]),
                   "+v"(o.v[2]));
      x += H.nb;
      const bool more = x < e;
      if (more && w == 0) hdr_commit<PREC>(g, R, L, hb ^ 1);
      typename BF::T* Fl = BF::at(L);
      if (one) {
        const int lane = __lane_id();
        if (lane < o.n) {
          Fl[w * BF::FSTRIDE + lane] = o.fx;
          Fl[w * BF::FSTRIDE + 64 + lane] = o.fy;
          Fl[w * BF::FSTRIDE + 128 + lane] = o.fz;
        }
      }
      __syncthreads();  // forces in LDS, staged entries free, next header complete
      if (one) {
        if (w == tw) fnb(H, o, (const typename BF::T*)Fl, BF::FSTRIDE);
      } else {
        fn(o);
      }
      if (!more) break;
      if (w != tw) stage_entries<PREC, WAVES - 1>(g, cells, hb ^ 1, L, (w + WAVES - 1 - tw) & (WAVES - 1));
      if (w == 0 && x + L.hb[hb ^ 1].nb < e) issue(x + L.hb[hb ^ 1].nb, R);
      hb ^= 1;
      nblk++;
    }
    return;
  }
  while (true) {
    __syncthreads();  // every wave is done with the previous block's LDS; header hb is complete
    const BlockHdr& H = L.hb[hb];
    const int tw = nblk & (WAVES - 1);
    const bool one = BTAIL && block_atoms(H) <= 64;
    ForceOut o;
    stage_fill<PREC>(g, cells, hb, L, o, OWN ? (one ? 2 : 1) : 0, tw);
    block_force<PREC, ENERGY, COUNT>(g, cells, H, L, o);
    if (OWN) {
      // the pair loop has covered the own cell's loads; from here on their values count
      // as plain registers, so the tail does not wait for the next block's count loads
      // (issued just before it) on their account
      asm volatile("" : "+v"(o.id), "+v"(o.x[0]), "+v"(o.x[1]), "+v"(o.x[2]), "+v"(o.v[0]), "+v"(o.v[1]),
                   "+v"(o.v[2]));
    }
    x += H.nb;
    const bool more = x < e;
    if (more && w == 0) issue(x, R);
    if (one) {
      typedef BlockForces<PREC> BF;
      typename BF::T* Fl = BF::at(L);
      const int lane = __lane_id();
      if (BF::AFTER_ALL) __syncthreads();  // every pair loop is done with the staged entries
      if (lane < o.n) {
        Fl[w * BF::FSTRIDE + lane] = (typename BF::T)o.fx;
        Fl[w * BF::FSTRIDE + 64 + lane] = (typename BF::T)o.fy;
        Fl[w * BF::FSTRIDE + 128 + lane] = (typename BF::T)o.fz;
      }
      __syncthreads();
      if (w == tw) fnb(H, o, (const typename BF::T*)Fl, BF::FSTRIDE);
    } else {
      fn(o);
    }
    if (!more) break;
    // the other header is free: every wave finished the block that used it before the
    // barrier above
    if (w == 0) hdr_commit<PREC>(g, R, L, hb ^ 1);
    hb ^= 1;
    nblk++;
  }
}

// Per-item accumulators of one wave.
struct ItemAcc {
  double u, w, k;                 // per lane (energy steps)
  double kt;                      // per lane: kinetic energy of v(t) (thermostat)
  unsigned nt;                    // per lane: atoms (thermostat)
  unsigned long long cand, inr;   // per lane (count mode)
  unsigned left, right;           // uniform migration counts
};

__device__ __forceinline__ void acc_zero(ItemAcc& a) {
  a.u = a.w = a.k = a.kt = 0.0;
  a.nt = 0;
  a.cand = a.inr = 0;
  a.left = a.right = 0;
}

// ---------------------------------------------------------------------------
// Velocity-Verlet + migration of one cell after its forces (kernels md_v3aa, md_v3b).
// The stored velocity is the half-step velocity v(t - dt/2), or v(t) itself on the
// first step after a load.  One step of the synchronous form:
//   v(t) = v(t-dt/2) + (dt/2) F(t);  v(t+dt/2) = v(t) + (dt/2) F(t);
//   r(t+dt) = r(t) + dt v(t+dt/2), wrapped; the new cell decides where the atom is
// stored: the same cell (kept in order), or appended to another cell -- possibly in
// the left or right neighbour slice.
// ---------------------------------------------------------------------------
// The update of one atom: v(t) (vf), v(t + dt/2) (vh), the wrapped r(t + dt) (xn), its
// cell coordinates (gc) and index (dest), slice move (dir: 0 none, 1 left, 2 right); error
// bits in bad.
// SCALE: the thermostat factor lam multiplies v(t) first.
template <bool SCALE>
__device__ __forceinline__ void advance(const DGeom& g, const double F[3], const double x[3], const double v[3],
                                        int first, double lam, int s_old, double vf[3], double vh[3],
                                        double xn[3], int gc[3], int& dest, int& dir, uint32_t& bad) {
#pragma unroll
  for (int d = 0; d < 3; d++) {
    vf[d] = first ? v[d] : add_rn(v[d], mul_rn(g.hdt, F[d]));
    if (SCALE) vf[d] = mul_rn(lam, vf[d]);
  }
#pragma unroll
  for (int d = 0; d < 3; d++) {
    vh[d] = add_rn(vf[d], mul_rn(g.hdt, F[d]));
    const double xs = add_rn(x[d], mul_rn(g.dt, vh[d]));
    xn[d] = wrap1(xs, g.L[d]);
    // NaN and infinite positions fail one of the two tests, and a non-finite velocity
    // always gives a non-finite position (dt is finite and positive)
    if (!(xn[d] >= 0.0) || xn[d] > g.L[d]) bad |= ERR_NONFINITE;
    gc[d] = coord_cell(xn[d], g.inv_l[d], g.G[d]);
  }
  const int s_new = qdiv(gc[0], g.inv_ncx);
  dest = s_new * g.cps + ((gc[0] - s_new * g.ncx) * g.G[1] + gc[1]) * g.G[2] + gc[2];
  int delta = s_new - s_old;  // both in [0, S): (s_new - s_old) mod S
  if (delta < 0) delta += g.S;
  if (delta == 1) dir = 2;
  else if (delta == g.S - 1) dir = 1;
  else if (delta != 0) bad |= ERR_DISPLACEMENT;
}

// Store of one updated atom: a stayer at its rank among the cell's stayers (id order
// kept), a mover appended from the top slot of its new cell.
template <int PREC>
__device__ __forceinline__ void store_atom(const RunArgs& ra, int dst, uint32_t* abort_flag, bool stay, bool ok,
                                           int rank, int dest, const double xn[3], const int gc[3],
                                           const double vh[3], uint32_t id) {
  int slot = -1;
  if (stay) {
    slot = rank;
  } else if (ok) {
    const unsigned old =
        __hip_atomic_fetch_add(gptr(ra.nin[dst]) + dest, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old < (unsigned)CELL_CAP) slot = CELL_CAP - 1 - (int)old;
    else raise_error(ra.err, abort_flag, ERR_CAPACITY);
  }
  if (slot >= 0) {
    gdouble* ob = cblk(ra.cells[dst], dest);
#pragma unroll
    for (int d = 0; d < 3; d++) {
      ob[d * CELL_CAP + slot] = xn[d];
      ob[(3 + d) * CELL_CAP + slot] = vh[d];
    }
    // the FP32 corner-relative copy only where the FP32 pair path reads it
    if constexpr (PREC == 1)
      crel(ob)[slot] = vf4{corner_rel(xn[0], gc[0], ra.g.l[0]), corner_rel(xn[1], gc[1], ra.g.l[1]),
                           corner_rel(xn[2], gc[2], ra.g.l[2]), 0.0f};
    cids(ob)[slot] = id;
  }
}

// One cell per wave (lanes < o.n).  SCALE: the thermostat factor lam multiplies v(t)
// first (the forces come from the thermostat's force pass; energies were sampled there).
template <int PREC, bool ENERGY, bool COUNT, bool SCALE>
__device__ void p2_tail(const RunArgs& ra, const ForceOut& o, int src, int s_old, int first, ItemAcc& acc,
                        uint32_t* abort_flag, double lam) {
  const DGeom& g = ra.g;
  const int lane = __lane_id();
  const int dst = src ^ 1;
  const int c = o.c;
  if (c < 0) return;
  if (o.n == 0) {
    if (lane == 0) gptr(ra.ncnt[dst])[c] = 0u;
    return;
  }
  const bool own = lane < o.n;
  double xn[3] = {0, 0, 0}, vh[3] = {0, 0, 0};
  int gc[3] = {0, 0, 0};
  int dest = c;
  uint32_t bad = 0;
  int dir = 0;
  if (own) {
    const double F[3] = {o.fx, o.fy, o.fz};
    double vf[3];
    advance<SCALE>(g, F, o.x, o.v, first, lam, s_old, vf, vh, xn, gc, dest, dir, bad);
    if (ENERGY) {
      acc.k += 0.5 * add_rn(add_rn(mul_rn(vf[0], vf[0]), mul_rn(vf[1], vf[1])),
                               mul_rn(vf[2], vf[2]));
      acc.u += o.uh;
      acc.w += o.wh;
    }
    if (COUNT) {
      acc.cand += (unsigned long long)(o.total - 1);
      acc.inr += o.pc;
    }
  }
  if (bad) raise_error(ra.err, abort_flag, bad);
  const bool ok = own && !bad;
  const bool stay = ok && dest == c;
  const unsigned long long sm = __ballot(stay);
  const int rank = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(sm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)sm, 0u));
  store_atom<PREC>(ra, dst, abort_flag, stay, ok, rank, dest, xn, gc, vh, own ? o.id : 0u);
  if (lane == 0) gptr(ra.ncnt[dst])[c] = (uint32_t)__popcll(sm);
  acc.left += (unsigned)__popcll(__ballot(ok && dir == 1));
  acc.right += (unsigned)__popcll(__ballot(ok && dir == 2));
}

// All cells of a block on one wave (plain steps): lane l holds atom l of the block's cells
// taken in order (at most 64 atoms), with its force F; cell q of the block holds lanes
// [P_q, P_q + n_q).  The same updates and stores as one p2_tail per cell.
template <int PREC, class T>
__device__ void p2_tail_block(const RunArgs& ra, const BlockHdr& H, const ForceOut& o, const T* Fl, int fstride,
                              int src, int s_old, int first, ItemAcc& acc, uint32_t* abort_flag) {
  const DGeom& g = ra.g;
  const int lane = __lane_id();
  const int dst = src ^ 1;
  int n[BZ], P[BZ + 1];
  P[0] = 0;
#pragma unroll
  for (int q = 0; q < BZ; q++) {
    n[q] = q < H.nb ? H.cnt[9 * (q + 1) + 4] : 0;
    P[q + 1] = P[q] + n[q];
  }
  static_assert(BZ == 4, "the cell split below assumes four cells per block");
  const int q = (lane >= P[1] ? 1 : 0) + (lane >= P[2] ? 1 : 0) + (lane >= P[3] ? 1 : 0);
  const int pq = q == 0 ? 0 : (q == 1 ? P[1] : (q == 2 ? P[2] : P[3]));
  const int c = H.nb_cell[9 * (q + 1) + 4];
  const bool own = lane < P[BZ];
  double xn[3] = {0, 0, 0}, vh[3] = {0, 0, 0};
  int gc[3] = {0, 0, 0};
  int dest = c;
  uint32_t bad = 0;
  int dir = 0;
  if (own) {
    // force of atom lane - pq of cell q, left in LDS by wave q
    const T* fq = Fl + q * fstride + lane - pq;
    const double F[3] = {(double)fq[0], (double)fq[64], (double)fq[128]};
    double vf[3];
    advance<false>(g, F, o.x, o.v, first, 1.0, s_old, vf, vh, xn, gc, dest, dir, bad);
  }
  if (bad) raise_error(ra.err, abort_flag, bad);
  const bool ok = own && !bad;
  const bool stay = ok && dest == c;
  const unsigned long long sm = __ballot(stay);
  // rank among the stayers of the lane's own cell: stayers below the lane minus those below
  // the cell's first lane
  const unsigned long long below_cell = pq == 0 ? 0ull : (sm & ((1ull << pq) - 1ull));
  const int rank =
      (int)__builtin_amdgcn_mbcnt_hi((unsigned)(sm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)sm, 0u)) -
      __popcll(below_cell);
  store_atom<PREC>(ra, dst, abort_flag, stay, ok, rank, dest, xn, gc, vh, own ? o.id : 0u);
  if (lane < H.nb) {
    // stayers of cell lane: the new count of its own slots
    const int pl = lane == 0 ? 0 : (lane == 1 ? P[1] : (lane == 2 ? P[2] : P[3]));
    const int nl = lane == 0 ? n[0] : (lane == 1 ? n[1] : (lane == 2 ? n[2] : n[3]));
    const unsigned long long seg = nl == 0 ? 0ull : ((nl == 64 ? ~0ull : ((1ull << nl) - 1ull)) << pl);
    gptr(ra.ncnt[dst])[H.nb_cell[9 * (lane + 1) + 4]] = (uint32_t)__popcll(sm & seg);
  }
  acc.left += (unsigned)__popcll(__ballot(ok && dir == 1));
  acc.right += (unsigned)__popcll(__ballot(ok && dir == 2));
}

// Force pass of a thermostat step (kernels md_v3a, md_v3aa, md_thermo_a): v(t) of
// every atom of the cell enters the slice's kinetic energy; F(t) is kept for the
// integrate pass, which runs once the whole slice is known (its scale factor needs
// every atom of the slice).
template <bool ENERGY, bool COUNT>
__device__ void p2_force_tail(const RunArgs& ra, const ForceOut& o, int src, int first, ItemAcc& acc) {
  const DGeom& g = ra.g;
  const int lane = __lane_id();
  const int c = o.c;
  if (c < 0 || lane >= o.n) return;
  const double F[3] = {o.fx, o.fy, o.fz};
  double vf[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const double v = o.v[d];
    vf[d] = first ? v : add_rn(v, mul_rn(g.hdt, F[d]));
  }
  const double ke =
      0.5 * add_rn(add_rn(mul_rn(vf[0], vf[0]), mul_rn(vf[1], vf[1])), mul_rn(vf[2], vf[2]));
  acc.kt += ke;
  acc.nt += 1u;
  if (ENERGY) {
    acc.k += ke;
    acc.u += o.uh;
    acc.w += o.wh;
  }
  if (COUNT) {
    acc.cand += (unsigned long long)(o.total - 1);
    acc.inr += o.pc;
  }
  double* fb = ra.fbuf + (size_t)c * 3 * CELL_CAP;
  fb[lane] = F[0];
  fb[CELL_CAP + lane] = F[1];
  fb[2 * CELL_CAP + lane] = F[2];
}

// ---------------------------------------------------------------------------
// Order the atoms of one cell by id (wave-wide rank sort).  Entries come from slots
// [0, n_low) and from the top slots [CAP - n_high, CAP); the result fills slots
// [0, n_low + n_high).  Every lane reads its entry before any lane writes.
// ---------------------------------------------------------------------------
__device__ void cell_sort_wave(unsigned char* cells, int c, int n_low, int n_high) {
  const int lane = __lane_id();
  const int n = n_low + n_high;
  gdouble* p = cblk(cells, c);
  guint32* ids = cids(p);
  const bool act = lane < n;
  const int from = lane < n_low ? lane : CELL_CAP - 1 - (lane - n_low);
  double v[6];
  vf4 r = {0.0f, 0.0f, 0.0f, 0.0f};
  uint32_t id = 0xffffffffu;
  if (act) {
#pragma unroll
    for (int d = 0; d < 6; d++) v[d] = p[d * CELL_CAP + from];
    r = crel(p)[from];
    id = ids[from];
  }
  int rank = 0;
  for (int m = 0; m < n; m++) {
    const uint32_t other = (uint32_t)__shfl((int)id, m);
    rank += other < id ? 1 : 0;
  }
  __asm__ volatile("" ::: "memory");
  wave_sync();
  if (act) {
#pragma unroll
    for (int d = 0; d < 6; d++) p[d * CELL_CAP + rank] = v[d];
    crel(p)[rank] = r;
    ids[rank] = id;
  }
}

// Finalise the cells [b, e) of one slice for the step held in parity `dst`: append the
// atoms that moved in, restore id order, publish the count; clear the move-in counters
// of the other parity for the next step.
__device__ void p1_range(const RunArgs& ra, int b, int e, int dst, int wave, uint32_t* abort_flag) {
  const int lane = __lane_id();
  const int src = dst ^ 1;
  for (int base = b + wave * 64; base < e; base += WAVES * 64) {
    const int c = base + lane;
    unsigned n_stay = 0, n_in = 0;
    if (c < e) {
      n_stay = gptr(ra.ncnt[dst])[c];
      // move-in counters are only ever accessed atomically (they are incremented by the
      // integrate items of this and the neighbouring slices, possibly on another XCD)
      n_in = __hip_atomic_load(gptr(ra.nin[dst]) + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(gptr(ra.nin[src]) + c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (n_stay + n_in > (unsigned)ra.g.cap) {
        raise_error(ra.err, abort_flag, ERR_CAPACITY);
        n_in = 0;
      }
      if (n_in) gptr(ra.ncnt[dst])[c] = n_stay + n_in;
    }
    unsigned long long dirty = __ballot(n_in != 0);
    while (dirty) {
      const int l = __ffsll((long long)dirty) - 1;
      dirty &= dirty - 1;
      const int cc = __shfl(c, l);
      const int lo = __shfl((int)n_stay, l);
      const int hi = __shfl((int)n_in, l);
      cell_sort_wave(ra.cells[dst], cc, lo, hi);
    }
  }
}

// ---------------------------------------------------------------------------
// Persistent kernel.
//   force/integrate item (phase 0) of slice i at step k needs the finalise items of
//   slices i-1, i, i+1 for step k; the finalise item (phase 1) of slice i for step
//   k+1 needs the force/integrate items of i-1, i, i+1 at step k.
// Two schedulers share the item bodies:
//   dataflow (default): the item that completes a dependency set appends the now
//     ready items to a queue; workers take queue slots in order, so nobody holds an
//     item whose inputs are missing;
//   ticket: items are dealt in a fixed per-step order (claim-order tables) and wait
//     on the per-slice counters of their neighbours.
// Both end: every item is pushed (dealt) exactly once and its dependencies were
// pushed (dealt) before it.
// ---------------------------------------------------------------------------
struct Item {
  int run, k, phase, slice, chunk, go;
};

// phase: 0 force (+ integrate without the thermostat), 1 finalise, 2 thermostat integrate
__device__ __forceinline__ unsigned long long enc_item(int run, int k, int phase, int slice, int chunk) {
  return (1ull << 63) | ((unsigned long long)run << 48) | ((unsigned long long)k << 29) |
         ((unsigned long long)phase << 27) | ((unsigned long long)slice << 12) | (unsigned long long)chunk;
}

__device__ __forceinline__ void dec_item(unsigned long long v, Item& it) {
  it.run = (int)((v >> 48) & 0x7fffull);
  it.k = (int)((v >> 29) & 0x7ffffull);
  it.phase = (int)((v >> 27) & 3ull);
  it.slice = (int)((v >> 12) & 0x7fffull);
  it.chunk = (int)(v & 0xfffull);
}

// Polls with relaxed loads (an acquire per poll would invalidate this XCD's L2 each
// time); the caller issues one acquire fence once the counters are reached.
__device__ bool wait_counters(const LaunchArgs& la, const uint32_t* cnt, int S, int s, unsigned need,
                              uint32_t* err, uint32_t* abort_flag) {
  const long long t_begin = wall_clock64();
  const int nb[3] = {(s + S - 1) % S, s, (s + 1) % S};
  for (int q = 0; q < 3; q++) {
    while (ld_relaxed(cnt + nb[q]) < need) {
      if (ld_relaxed(abort_flag)) return false;
      if (wall_clock64() - t_begin > la.watchdog_ticks) {
        raise_error(err, abort_flag, ERR_WATCHDOG);
        return false;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  return true;
}

// Force item of slice i at step k (Algorithm 1 over the item's cells).  NVT: forces
// and the kinetic energy of v(t) only; the integrate item follows.  Otherwise the
// velocity-Verlet update and migration follow at once, cell by cell.
template <int PREC, bool ENERGY, bool COUNT, bool NVT>
__device__ void run_p2_item(const RunArgs& ra, const Item& it, BlockLDS<PREC>& L, double (*s_red)[4],
                            unsigned long long (*s_cnt)[5], uint32_t* abort_flag) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int src = (ra.par0 + it.k) & 1;
  const int first = (it.k == 0) ? ra.first : 0;
  const int b = (int)((long long)ra.g.cps * it.chunk / ra.nch);
  const int e = (int)((long long)ra.g.cps * (it.chunk + 1) / ra.nch);
  ItemAcc acc;
  acc_zero(acc);
  // plain steps finish a block on one wave; energy, count and thermostat steps per wave
  constexpr bool BTAIL = !ENERGY && !COUNT && !NVT;
  for_blocks<PREC, ENERGY, COUNT, true, BTAIL>(
      ra.g, ra.cells[src], ra.ncnt[src], it.slice, b, e, L,
      [&](const ForceOut& o) {
        if (NVT) p2_force_tail<ENERGY, COUNT>(ra, o, src, first, acc);
        else p2_tail<PREC, ENERGY, COUNT, false>(ra, o, src, it.slice, first, acc, abort_flag, 1.0);
      },
      [&](const BlockHdr& H, const ForceOut& o, const auto* Fl, int fstride) {
        p2_tail_block<PREC>(ra, H, o, Fl, fstride, src, it.slice, first, acc, abort_flag);
      });
  // wave reductions (fixed butterfly), then waves in order
  double u = acc.u, w = acc.w, k = acc.k, kt = acc.kt;
  unsigned long long cc = acc.cand, pc = acc.inr, nt = acc.nt;
  if (ENERGY || COUNT || NVT) {
    for (int off = 32; off >= 1; off >>= 1) {
      if (ENERGY) {
        u += __shfl_xor(u, off);
        w += __shfl_xor(w, off);
        k += __shfl_xor(k, off);
      }
      if (COUNT) {
        cc += __shfl_xor(cc, off);
        pc += __shfl_xor(pc, off);
      }
      if (NVT) {
        kt += __shfl_xor(kt, off);
        nt += __shfl_xor(nt, off);
      }
    }
  }
  if (lane == 0) {
    s_red[wave][0] = u;
    s_red[wave][1] = k;
    s_red[wave][2] = w;
    s_red[wave][3] = kt;
    s_cnt[wave][0] = acc.left;
    s_cnt[wave][1] = acc.right;
    s_cnt[wave][2] = cc;
    s_cnt[wave][3] = pc;
    s_cnt[wave][4] = nt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long t = ra.t0 + it.k;
    if (ENERGY) {
      const long long j = t / ra.every - (ra.t0 + ra.every - 1) / ra.every;
      double su = 0, sk = 0, sw = 0;
      for (int q = 0; q < WAVES; q++) {
        su += s_red[q][0];
        sk += s_red[q][1];
        sw += s_red[q][2];
      }
      double* ep = ra.epart + ((j * ra.g.S + it.slice) * ra.nch + it.chunk) * 3;
      ep[0] = su;
      ep[1] = sk;
      ep[2] = sw;
    }
    if (NVT) {
      double skt = 0;
      unsigned long long snt = 0;
      for (int q = 0; q < WAVES; q++) {
        skt += s_red[q][3];
        snt += s_cnt[q][4];
      }
      double* kp = ra.kpart + ((size_t)it.slice * ra.nch + it.chunk) * 2;
      kp[0] = skt;
      kp[1] = (double)snt;
    }
    unsigned long long left = 0, right = 0, c2 = 0, p2 = 0;
    for (int q = 0; q < WAVES; q++) {
      left += s_cnt[q][0];
      right += s_cnt[q][1];
      c2 += s_cnt[q][2];
      p2 += s_cnt[q][3];
    }
    if (left) atomicAdd(ra.migcum + 2 * it.slice + 0, left);
    if (right) atomicAdd(ra.migcum + 2 * it.slice + 1, right);
    if (ra.miglog) {
      if (left) atomicAdd(ra.miglog + ((size_t)it.k * ra.g.S + it.slice) * 2 + 0, (uint32_t)left);
      if (right) atomicAdd(ra.miglog + ((size_t)it.k * ra.g.S + it.slice) * 2 + 1, (uint32_t)right);
    }
    if (COUNT) {
      atomicAdd(ra.paircnt + 0, c2);
      atomicAdd(ra.paircnt + 1, p2);
    }
    if (ra.fail_at >= 0 && t == ra.fail_at && it.slice == 0 && it.chunk == 0)
      raise_error(ra.err, abort_flag, ERR_INJECTED);
  }
}

// Integrate item of a thermostat step (kernels md_thermo_b, md_v3b): the slice's scale
// factor from the kinetic energy of all its force items (summed in chunk order), then
// the velocity-Verlet update with v(t) scaled, and migration, cell by cell.
template <int PREC>
__device__ void run_p2b_item(const RunArgs& ra, const Item& it, double* s_lam, unsigned long long (*s_cnt)[5],
                             uint32_t* abort_flag) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int src = (ra.par0 + it.k) & 1;
  const int first = (it.k == 0) ? ra.first : 0;
  if (threadIdx.x == 0) {
    double K = 0.0, n = 0.0;
    const double* kp = ra.kpart + (size_t)it.slice * ra.nch * 2;
    for (int ch = 0; ch < ra.nch; ch++) {
      K += kp[2 * ch];
      n += kp[2 * ch + 1];
    }
    *s_lam = (n > 0.0 && K > 0.0) ? __dsqrt_rn(__ddiv_rn(mul_rn(mul_rn(3.0, n), ra.thermo_T), mul_rn(2.0, K)))
                                  : 1.0;
  }
  __syncthreads();
  const double lam = *s_lam;
  const int b = (int)((long long)ra.g.cps * it.chunk / ra.nch);
  const int e = (int)((long long)ra.g.cps * (it.chunk + 1) / ra.nch);
  const int cbase = it.slice * ra.g.cps;
  ItemAcc acc;
  acc_zero(acc);
  for (int c = cbase + b + wave; c < cbase + e; c += WAVES) {
    ForceOut o;
    o.c = c;
    o.n = (int)gptr(ra.ncnt[src])[c];
    o.total = 0;
    o.pc = 0;
    o.uh = o.wh = 0.0;
    o.fx = o.fy = o.fz = 0.0;
    if (lane < o.n) {
      const double* fb = ra.fbuf + (size_t)c * 3 * CELL_CAP;
      o.fx = fb[lane];
      o.fy = fb[CELL_CAP + lane];
      o.fz = fb[2 * CELL_CAP + lane];
      const gdouble* ib = cblk(ra.cells[src], c);
#pragma unroll
      for (int d = 0; d < 3; d++) {
        o.x[d] = ib[d * CELL_CAP + lane];
        o.v[d] = ib[(3 + d) * CELL_CAP + lane];
      }
      o.id = cids(ib)[lane];
    }
    p2_tail<PREC, false, false, true>(ra, o, src, it.slice, first, acc, abort_flag, lam);
  }
  if (lane == 0) {
    s_cnt[wave][0] = acc.left;
    s_cnt[wave][1] = acc.right;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long left = 0, right = 0;
    for (int q = 0; q < WAVES; q++) {
      left += s_cnt[q][0];
      right += s_cnt[q][1];
    }
    if (left) atomicAdd(ra.migcum + 2 * it.slice + 0, left);
    if (right) atomicAdd(ra.migcum + 2 * it.slice + 1, right);
    if (ra.miglog) {
      if (left) atomicAdd(ra.miglog + ((size_t)it.k * ra.g.S + it.slice) * 2 + 0, (uint32_t)left);
      if (right) atomicAdd(ra.miglog + ((size_t)it.k * ra.g.S + it.slice) * 2 + 1, (uint32_t)right);
    }
  }
}

// KIND: 0 plain steps only; 1 also energy-sampled steps; 2 also pair counting (the
// variants differ in register needs, and a kernel is allocated for its largest path).
// NVT: the kernel variant that also runs thermostat steps (ra.thermo_T > 0).
template <int PREC, int KIND, bool NVT>
__device__ void run_item(const RunArgs& ra, const Item& it, BlockLDS<PREC>& ws, double (*s_red)[4],
                         unsigned long long (*s_cnt)[5]) {
  const int wave = threadIdx.x >> 6;
  const bool nvt = NVT && ra.thermo_T > 0.0;
  if (it.phase == 0) {
    const long long t = ra.t0 + it.k;
    const bool energy = ra.every > 0 && (t % ra.every) == 0;
    if (KIND == 0) {
      if (NVT && nvt) run_p2_item<PREC, false, false, NVT>(ra, it, ws, s_red, s_cnt, ra.abort);
      else run_p2_item<PREC, false, false, false>(ra, it, ws, s_red, s_cnt, ra.abort);
    } else if (KIND == 1) {
      if (NVT && nvt) {
        if (energy) run_p2_item<PREC, true, false, NVT>(ra, it, ws, s_red, s_cnt, ra.abort);
        else run_p2_item<PREC, false, false, NVT>(ra, it, ws, s_red, s_cnt, ra.abort);
      } else {
        if (energy) run_p2_item<PREC, true, false, false>(ra, it, ws, s_red, s_cnt, ra.abort);
        else run_p2_item<PREC, false, false, false>(ra, it, ws, s_red, s_cnt, ra.abort);
      }
    } else if (NVT && nvt) {
      if (ra.count) {
        if (energy) run_p2_item<PREC, true, true, NVT>(ra, it, ws, s_red, s_cnt, ra.abort);
        else run_p2_item<PREC, false, true, NVT>(ra, it, ws, s_red, s_cnt, ra.abort);
      } else {
        if (energy) run_p2_item<PREC, true, false, NVT>(ra, it, ws, s_red, s_cnt, ra.abort);
        else run_p2_item<PREC, false, false, NVT>(ra, it, ws, s_red, s_cnt, ra.abort);
      }
    } else if (ra.count) {
      if (energy) run_p2_item<PREC, true, true, false>(ra, it, ws, s_red, s_cnt, ra.abort);
      else run_p2_item<PREC, false, true, false>(ra, it, ws, s_red, s_cnt, ra.abort);
    } else {
      if (energy) run_p2_item<PREC, true, false, false>(ra, it, ws, s_red, s_cnt, ra.abort);
      else run_p2_item<PREC, false, false, false>(ra, it, ws, s_red, s_cnt, ra.abort);
    }
  } else if (NVT && it.phase == 2) {
    run_p2b_item<PREC>(ra, it, &s_red[0][0], s_cnt, ra.abort);
  } else {
    const int dst = (ra.par0 + it.k + 1) & 1;
    const int b = (int)((long long)ra.g.cps * it.chunk / ra.nchA);
    const int e = (int)((long long)ra.g.cps * (it.chunk + 1) / ra.nchA);
    const int cbase = it.slice * ra.g.cps;
    p1_range(ra, cbase + b, cbase + e, dst, wave, ra.abort);
  }
}

// Append the n chunks of item (run, k, phase, slice) to the queue of the slice (thread 0
// of the item whose completion made the dependency set complete).  The pusher first
// acquires (every counted item released before its increment) and releases, so whoever
// takes the items sees the results of all the counted items.
__device__ void push_items(const LaunchArgs& la, const RunArgs& ra, int run, int k, int phase, int slice,
                           int n) {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
  const int x = la.nq > 1 ? slice_queue(ra, la.nq, slice) : 0;
  const long long room = la.qoff[x + 1] - la.qoff[x];
  const unsigned long long base = __hip_atomic_fetch_add(gptr(la.q_tail) + XQ_STRIDE * x,
                                                         (unsigned long long)n, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
  if ((long long)base + n > room) {  // never expected: the host sized every queue exactly
    raise_error(la.launch_err, nullptr, ERR_BADINPUT);
    return;
  }
  for (int ch = 0; ch < n; ch++)
    __hip_atomic_store(gptr(la.q) + la.qoff[x] + base + ch, enc_item(run, k, phase, slice, ch),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Dataflow completion (thread 0, after the item's release fence): count this item
// towards its dependents with relaxed increments; the count that completes a dependency
// set acquires (every counted item released before its increment), releases, and
// appends the dependent items (all chunks) to the queue.
__device__ void complete_dataflow(const LaunchArgs& la, const RunArgs& ra, const Item& it) {
  const int S = ra.g.S;
  const bool nvt = ra.thermo_T > 0.0;
  if (nvt && it.phase == 0) {
    // thermostat: the slice's integrate items wait for all of its force items
    const unsigned needk = (unsigned)ra.nch * (unsigned)(it.k + 1);
    const unsigned old = __hip_atomic_fetch_add(gptr(ra.cntK) + it.slice, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1u != needk) return;
    push_items(la, ra, it.run, it.k, 2, it.slice, ra.nch);
    return;
  }
  // the step's update of slice i (phase 0, or 2 with the thermostat) counts towards the
  // finalise of i-1, i, i+1; a finalise counts towards the next force items
  const bool update = it.phase != 1;
  const unsigned need = 3u * (unsigned)(update ? ra.nch : ra.nchA) * (unsigned)(it.k + 1);
  uint32_t* cnt = update ? ra.cntF : ra.cntA;
  for (int d = -1; d <= 1; d++) {
    const int j = (it.slice + d + S) % S;
    const unsigned old = __hip_atomic_fetch_add(gptr(cnt) + j, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1u != need) continue;
    int phase, k;
    if (update) {
      phase = 1;  // finalise of step k+1
      k = it.k;
    } else {
      if (it.k + 1 >= ra.nsteps) continue;  // the launch ends with this finalise
      phase = 0;
      k = it.k + 1;
    }
    push_items(la, ra, it.run, k, phase, j, phase == 1 ? ra.nchA : ra.nch);
  }
}

// Whether an item ends with an agent-scope release.  Items exchange data through memory:
// an item's inputs are the cells (and counters) its dependencies wrote, its outputs are
// read by its dependents.  Every item starts with an agent-scope acquire (it invalidates
// the compute unit's L1; the L2 keeps its lines).  Its stores have completed in its XCD's
// L2 before it is counted (every wave waits for them).  With one queue for the device
// (nq = 1) its dependents may run on any XCD, so it also releases at agent scope: the
// XCD's L2 writes its dirty lines back, and other XCDs see them.  With XCD queues the
// items of a slice run on the XCD that owns it, and the items of slice i read and write
// only slices i-1, i, i+1: when all three belong to the same XCD, every dependent reads
// the item's outputs through the same L2 and the write-back is not needed.  A slice next
// to another XCD's range, or an item run by a workgroup that is not on the queue's XCD,
// releases at agent scope.  Move-in counters, incremented by neighbours' integrate items,
// are accessed atomically only.
__device__ __forceinline__ bool release_full(const LaunchArgs& la, const RunArgs& ra, const Item& it,
                                             bool own_xcd) {
  if (la.nq == 1 || !own_xcd) return true;
  const int S = ra.g.S;
  const int x = slice_queue(ra, la.nq, it.slice);
  return slice_queue(ra, la.nq, (it.slice + S - 1) % S) != x || slice_queue(ra, la.nq, (it.slice + 1) % S) != x;
}

// KIND (see run_item): 0 launches without energy samples or pair counting (fewest
// registers), 1 with energy samples, 2 with pair counting.  NVT: with a thermostat run.
template <int PREC, int KIND, bool NVT>
__device__ __forceinline__ void persistent_body(const LaunchArgs& la) {
  __shared__ BlockLDS<PREC> ws;
  __shared__ double s_red[WAVES][4];
  __shared__ unsigned long long s_cnt[WAVES][5];
  __shared__ Item s_it;
  __shared__ int s_ok;
  __shared__ int s_full;
  __shared__ long long s_ticket;
  __shared__ RunArgs s_ra;
  static_assert(sizeof(RunArgs) % 4 == 0, "RunArgs is copied as dwords");
  // the queue this workgroup serves: its XCD's (nq > 1); a workgroup on an XCD without a
  // queue of its own (never expected) serves one with agent-scope fences on every item
  const int xq_hw = la.nq > 1 ? xcc_id() : 0;
  const int xq = xq_hw % la.nq;
  const bool own_xcd = la.nq > 1 && xq_hw < la.nq;
  const long long qbase = la.qoff[xq];
  const long long total = la.qoff[xq + 1] - qbase;
  while (true) {
    if (threadIdx.x == 0) {
      Item it;
      it.go = 0;
      const long long T = (long long)__hip_atomic_fetch_add(gptr(la.ticket) + XQ_STRIDE * xq, 1ull,
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_ticket = qbase + T;  // the item's slot (and trace record)
      if (la.trace && T < total) la.trace[qbase + T].t_claim = wall_clock64();
      if (T < total) {
        if (la.mode == 0) {
          // dataflow: wait for slot T of the queue to be filled
          const long long t_begin = wall_clock64();
          unsigned long long v;
          // relaxed polling; the acquire fence follows once the item is known
          while (!((v = __hip_atomic_load(gptr(la.q) + qbase + T, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 63)) {
            if (ld_relaxed(la.launch_err)) break;
            if (wall_clock64() - t_begin > la.watchdog_ticks) {
              raise_error(la.launch_err, nullptr, ERR_WATCHDOG);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          if (v >> 63) {
            dec_item(v, it);
            it.go = 1;
          }
        } else {
          int lo = 0, hi = la.nrounds;
          while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (la.round_base[mid] <= T) lo = mid; else hi = mid;
          }
          const int k = lo;
          const long long rem = T - la.round_base[k];
          int rlo = 0, rhi = la.round_active[k];
          while (rhi - rlo > 1) {
            int mid = (rlo + rhi) >> 1;
            if (la.run_prefix[mid] <= rem) rlo = mid; else rhi = mid;
          }
          const RunArgs& ra = la.runs[rlo];
          const int local = (int)(rem - la.run_prefix[rlo]);
          // fixed claim orders: both phases have nch items per slice (nchA == nch); a round
          // holds wlev steps, the table gives each entry's step within the round
          const int entry = local / ra.nch;
          const unsigned ord = ra.order[entry];
          it.run = rlo;
          it.k = k * ra.wlev + (int)(ord >> 16);
          it.phase = (int)((ord >> 15) & 1u);
          it.slice = (int)(ord & 0x7fffu);
          it.chunk = local - entry * ra.nch;
          it.go = 1;
        }
      }
      s_it = it;
    }
    __syncthreads();
    const Item it = s_it;
    if (it.go == 0) break;
    // The item's run arguments, copied into LDS (they do not change during a launch):
    // read from global memory, every field would be loaded again after each store of
    // the item (the compiler must assume they may alias), each load waiting for all of
    // the wave's outstanding memory operations; LDS cannot alias global memory.
    {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(la.runs + it.run);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&s_ra);
      for (int i = threadIdx.x; i < (int)(sizeof(RunArgs) / 4); i += WG) dst[i] = src[i];
    }
    const RunArgs& rg = la.runs[it.run];  // thread 0 before the barrier below: the global copy
    if (threadIdx.x == 0) {
      bool ok = !ld_relaxed(rg.abort);
      if (la.mode != 0 && ok) {
        const unsigned need = (unsigned)(it.k + 1) * (unsigned)(it.phase == 0 ? rg.nchA : rg.nch);
        ok = wait_counters(la, it.phase == 0 ? rg.cntA : rg.cntF, rg.g.S, it.slice, need, rg.err, rg.abort);
      }
      // one acquire for the workgroup: the barrier below orders every wave after it
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_full = release_full(la, rg, it, own_xcd);
      s_ok = ok;
      if (la.trace) {
        TraceRec& tr = la.trace[s_ticket];
        tr.t_ready = wall_clock64();
        tr.k = (uint32_t)it.k;
        tr.slice = (uint32_t)it.slice;
        tr.chunk = (uint32_t)it.chunk;
        tr.phase = (uint32_t)it.phase;
        tr.hw_id = __smid();
        tr.launch = la.launch_index;
        tr.xcd = (uint32_t)xcc_id();
        tr.queue = (uint32_t)xq;
      }
    }
    __syncthreads();
    const RunArgs& ra = s_ra;  // after the barrier: the LDS copy
    const int ok = s_ok;
    if (ok) run_item<PREC, KIND, NVT>(ra, it, ws, s_red, s_cnt);
    // every wave's stores have reached the L2 before the barrier (the barrier itself
    // does not wait for them); thread 0's release then covers the whole workgroup
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
      if (s_full) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (la.trace) la.trace[s_ticket].t_done = wall_clock64();
      if (la.mode == 0) {
        // an aborted run still completes its items (without work) so the queue drains
        complete_dataflow(la, ra, it);
      } else if (ok) {
        uint32_t* cnt = it.phase == 0 ? ra.cntF : ra.cntA;
        __hip_atomic_fetch_add(gptr(cnt) + it.slice, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
  }
}

// The FP32 kernels for plain launches, launches with energy samples and thermostat
// launches are held to 128 VGPRs (4 waves per SIMD), the FP64 ones to 168 (3 waves per
// SIMD; FP64 workgroups need that much LDS anyway): a launch runs all its steps in one
// kernel, and the registers that a sampled or thermostat step would need beyond that are
// spilled on those steps rather than lowering the occupancy of every step.  The
// pair-counting (statistics) kernels and the thermostat kernels with energy samples take
// what they need.
#define MD_WPE(n) __attribute__((amdgpu_waves_per_eu(n)))
__global__ __launch_bounds__(WG) MD_WPE(4) void persistent_f32_lean(LaunchArgs la) { persistent_body<1, 0, false>(la); }
__global__ __launch_bounds__(WG) MD_WPE(4) void persistent_f32_energy(LaunchArgs la) { persistent_body<1, 1, false>(la); }
__global__ __launch_bounds__(WG) void persistent_f32_full(LaunchArgs la) { persistent_body<1, 2, false>(la); }
__global__ __launch_bounds__(WG) MD_WPE(3) void persistent_f64_lean(LaunchArgs la) { persistent_body<0, 0, false>(la); }
__global__ __launch_bounds__(WG) MD_WPE(3) void persistent_f64_energy(LaunchArgs la) { persistent_body<0, 1, false>(la); }
__global__ __launch_bounds__(WG) void persistent_f64_full(LaunchArgs la) { persistent_body<0, 2, false>(la); }
__global__ __launch_bounds__(WG) MD_WPE(4) void persistent_f32_lean_nvt(LaunchArgs la) { persistent_body<1, 0, true>(la); }
__global__ __launch_bounds__(WG) void persistent_f32_energy_nvt(LaunchArgs la) { persistent_body<1, 1, true>(la); }
__global__ __launch_bounds__(WG) void persistent_f32_full_nvt(LaunchArgs la) { persistent_body<1, 2, true>(la); }
__global__ __launch_bounds__(WG) MD_WPE(3) void persistent_f64_lean_nvt(LaunchArgs la) { persistent_body<0, 0, true>(la); }
__global__ __launch_bounds__(WG) void persistent_f64_energy_nvt(LaunchArgs la) { persistent_body<0, 1, true>(la); }
__global__ __launch_bounds__(WG) void persistent_f64_full_nvt(LaunchArgs la) { persistent_body<0, 2, true>(la); }
#undef MD_WPE

typedef void (*PersistentFn)(LaunchArgs);
static PersistentFn persistent_fn(int prec, int kind, int nvt) {
  static const PersistentFn fns[2][3][2] = {
      {{persistent_f64_lean, persistent_f64_lean_nvt},
       {persistent_f64_energy, persistent_f64_energy_nvt},
       {persistent_f64_full, persistent_f64_full_nvt}},
      {{persistent_f32_lean, persistent_f32_lean_nvt},
       {persistent_f32_energy, persistent_f32_energy_nvt},
       {persistent_f32_full, persistent_f32_full_nvt}}};
  return fns[prec == 1][kind < 0 ? 0 : (kind > 2 ? 2 : kind)][nvt != 0];
}

// Launch set-up: counters, abort flags, claim counter; in dataflow mode the queue holds
// the force/integrate items of the first step of every run.
__global__ void init_launch_kernel(LaunchArgs la) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  if (i < la.nq) {
    la.ticket[XQ_STRIDE * i] = 0ull;
    if (la.q_tail) la.q_tail[XQ_STRIDE * i] = (unsigned long long)la.prefill[i];
  }
  if (i == 0 && la.launch_err) *la.launch_err = 0u;
  for (int r = 0; r < la.nruns; r++) {
    const RunArgs& ra = la.runs[r];
    if (i == 0) {
      *ra.abort = 0u;
      *ra.err = 0u;
      ra.paircnt[0] = ra.paircnt[1] = 0ull;
    }
    for (long long s = i; s < ra.g.S; s += stride) {
      ra.cntA[s] = la.mode == 0 ? 0u : (uint32_t)ra.nchA;
      ra.cntF[s] = 0u;
      if (ra.cntK) ra.cntK[s] = 0u;
    }
    if (la.mode == 0 && ra.nsteps > 0) {
      // the first step's force items, each in its slice's queue (after the earlier runs')
      const long long n0 = (long long)ra.g.S * ra.nch;
      for (long long e = i; e < n0; e += stride) {
        const int s = (int)(e / ra.nch), ch = (int)(e % ra.nch);
        const int x = slice_queue(ra, la.nq, s);
        la.q[la.qoff[x] + ra.q0[x] + (long long)(s - ra.xfirst[x]) * ra.nch + ch] = enc_item(r, 0, 0, s, ch);
      }
    }
  }
}

// After a launch: every run's error word into one array (one copy for the host).
__global__ void gather_errors_kernel(const RunArgs* runs, int nruns, uint32_t* out) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nruns; r += gridDim.x * blockDim.x) out[r] = *runs[r].err;
}

// ---------------------------------------------------------------------------
// Load: bin every atom (Sec. 4 cell grid) and append it to its cell; then id order.
// ---------------------------------------------------------------------------
__global__ void fill_u32_kernel(uint32_t* p, long long n, uint32_t v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void load_scatter_kernel(DGeom g, const double* pos, const double* vel, long long n,
                                    unsigned char* cells, uint32_t* ncnt, uint32_t* err) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    int gc[3];
    for (int d = 0; d < 3; d++) gc[d] = coord_cell(pos[3 * i + d], g.inv_l[d], g.G[d]);
    const int c = global_cell(g, gc[0], gc[1], gc[2]);
    const unsigned slot = atomicAdd(ncnt + c, 1u);
    if (slot < (unsigned)g.cap) {
      gdouble* b = cblk(cells, c);
      for (int d = 0; d < 3; d++) {
        b[d * CELL_CAP + slot] = pos[3 * i + d];
        b[(3 + d) * CELL_CAP + slot] = vel[3 * i + d];
      }
      crel(b)[slot] = vf4{corner_rel(pos[3 * i], gc[0], g.l[0]), corner_rel(pos[3 * i + 1], gc[1], g.l[1]),
                          corner_rel(pos[3 * i + 2], gc[2], g.l[2]), 0.0f};
      cids(b)[slot] = (uint32_t)i;
    } else {
      atomicOr(err, ERR_CAPACITY);
    }
  }
}

__global__ __launch_bounds__(WG) void sort_cells_kernel(DGeom g, unsigned char* cells, uint32_t* ncnt,
                                                        uint32_t* err) {
  const int c = blockIdx.x * WAVES + (threadIdx.x >> 6);
  if (c >= g.ncell) return;
  unsigned n = ncnt[c];
  if (n > (unsigned)g.cap) {
    if ((threadIdx.x & 63) == 0) atomicOr(err, ERR_CAPACITY);
    return;
  }
  if (n > 1) cell_sort_wave(cells, c, (int)n, 0);
}

// ---------------------------------------------------------------------------
// Synchronous pass: F(t), v(t) and the energy terms at the current step, written in
// id order (md_get_state / md_energy_virial).
// ---------------------------------------------------------------------------
constexpr int SYNC_CELLS = 64;  // cells per workgroup of the synchronous pass

template <int PREC>
__global__ __launch_bounds__(WG) void sync_kernel(DGeom g, const unsigned char* cells,
                                                  const uint32_t* ncnt, int first, double* out_pos,
                                                  double* out_vel, double* out_force, double* epart,
                                                  uint32_t* err) {
  __shared__ BlockLDS<PREC> L;
  __shared__ double s_red[WAVES][3];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double u = 0, w = 0, k = 0;
  // SYNC_CELLS consecutive cells of one slice per workgroup
  const int per_slice = (g.cps + SYNC_CELLS - 1) / SYNC_CELLS;
  const int slice = blockIdx.x / per_slice;
  const int b = (blockIdx.x % per_slice) * SYNC_CELLS;
  const int e = min(g.cps, b + SYNC_CELLS);
  for_blocks<PREC, true, false, false, false>(g, cells, ncnt, slice, b, e, L, [&](const ForceOut& o) {
    if (o.c >= 0 && lane < o.n) {
      const gdouble* ib = cblk(cells, o.c);
      const uint32_t id = cids(ib)[lane];
      const double F[3] = {o.fx, o.fy, o.fz};
      double vf[3];
      for (int d = 0; d < 3; d++) {
        const double v = ib[(3 + d) * CELL_CAP + lane];
        vf[d] = first ? v : add_rn(v, mul_rn(g.hdt, F[d]));
        if (out_pos) out_pos[3 * (size_t)id + d] = ib[d * CELL_CAP + lane];
        if (out_vel) out_vel[3 * (size_t)id + d] = vf[d];
        if (out_force) out_force[3 * (size_t)id + d] = F[d];
        if (!isfinite(F[d]) || !isfinite(vf[d])) atomicOr(err, ERR_NONFINITE);
      }
      k += 0.5 * add_rn(add_rn(mul_rn(vf[0], vf[0]), mul_rn(vf[1], vf[1])),
                           mul_rn(vf[2], vf[2]));
      u += o.uh;
      w += o.wh;
    }
  }, [](const BlockHdr&, const ForceOut&, const auto*, int) {});
  for (int off = 32; off >= 1; off >>= 1) {
    u += __shfl_xor(u, off);
    w += __shfl_xor(w, off);
    k += __shfl_xor(k, off);
  }
  if (lane == 0) {
    s_red[wave][0] = u;
    s_red[wave][1] = k;
    s_red[wave][2] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double su = 0, sk = 0, sw = 0;
    for (int q = 0; q < WAVES; q++) {
      su += s_red[q][0];
      sk += s_red[q][1];
      sw += s_red[q][2];
    }
    epart[3 * blockIdx.x + 0] = su;
    epart[3 * blockIdx.x + 1] = sk;
    epart[3 * blockIdx.x + 2] = sw;
  }
}

__global__ void cells_of_kernel(DGeom g, const uint32_t* ncnt, const unsigned char* cells,
                                long long* cell_of_id) {
  const int c = blockIdx.x * WAVES + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= g.ncell) return;
  const unsigned n = ncnt[c];
  if ((unsigned)lane < n) cell_of_id[cids(cblk(cells, c))[lane]] = c;
}

__global__ void slice_counts_kernel(DGeom g, const uint32_t* ncnt, unsigned long long* counts) {
  const int s = blockIdx.x;
  unsigned long long acc = 0;
  for (int c = threadIdx.x; c < g.cps; c += blockDim.x) acc += ncnt[(size_t)s * g.cps + c];
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  __shared__ unsigned long long part[WAVES];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < WAVES; q++) t += part[q];
    counts[s] = t;
  }
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------
static inline hipStream_t S_(void* s) { return reinterpret_cast<hipStream_t>(s); }

static int grid_for(long long n, int block) {
  long long b = (n + block - 1) / block;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (int)b;
}

int launch_clear_u32(uint32_t* p, long long n, uint32_t value, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, S_(stream), p, n, value);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_load_scatter(const DGeom& g, const double* pos, const double* vel, long long n,
                        unsigned char* cells, uint32_t* ncnt, uint32_t* err, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(load_scatter_kernel, dim3(grid_for(n, 256)), dim3(256), 0, S_(stream), g, pos,
                     vel, n, cells, ncnt, err);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_sort_cells(const DGeom& g, unsigned char* cells, uint32_t* ncnt, uint32_t* err, void* stream) {
  const int blocks = (g.ncell + WAVES - 1) / WAVES;
  hipLaunchKernelGGL(sort_cells_kernel, dim3(blocks), dim3(WG), 0, S_(stream), g, cells, ncnt, err);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_init(const LaunchArgs& la, long long work, void* stream) {
  hipLaunchKernelGGL(init_launch_kernel, dim3(grid_for(work, 256)), dim3(256), 0, S_(stream), la);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int persistent_grid(int prec, int kind, int nvt, int* blocks_per_cu, int* cus) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return -1;
  int nb = 0;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persistent_fn(prec, kind, nvt), WG, 0);
  if (e != hipSuccess || nb < 1) nb = 1;
  *blocks_per_cu = nb;
  *cus = prop.multiProcessorCount;
  return 0;
}

int launch_gather_errors(const RunArgs* runs, int nruns, uint32_t* out, void* stream) {
  if (nruns <= 0) return 0;
  hipLaunchKernelGGL(gather_errors_kernel, dim3(grid_for(nruns, 256)), dim3(256), 0, S_(stream), runs, nruns, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_persistent(const LaunchArgs& la, int prec, int kind, int nvt, int grid, void* stream) {
  hipLaunchKernelGGL(persistent_fn(prec, kind, nvt), dim3(grid), dim3(WG), 0, S_(stream), la);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int sync_blocks(const DGeom& g) { return g.S * ((g.cps + SYNC_CELLS - 1) / SYNC_CELLS); }

int launch_sync(const DGeom& g, const unsigned char* cells, const uint32_t* ncnt, int first,
                double* out_pos, double* out_vel, double* out_force, double* epart, uint32_t* err,
                void* stream) {
  const int blocks = sync_blocks(g);
  if (g.prec == 1)
    hipLaunchKernelGGL(sync_kernel<1>, dim3(blocks), dim3(WG), 0, S_(stream), g, cells, ncnt, first,
                       out_pos, out_vel, out_force, epart, err);
  else
    hipLaunchKernelGGL(sync_kernel<0>, dim3(blocks), dim3(WG), 0, S_(stream), g, cells, ncnt, first,
                       out_pos, out_vel, out_force, epart, err);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_cells_of(const DGeom& g, const uint32_t* ncnt, const unsigned char* cells,
                    long long* cell_of_id, void* stream) {
  const int blocks = (g.ncell + WAVES - 1) / WAVES;
  hipLaunchKernelGGL(cells_of_kernel, dim3(blocks), dim3(WG), 0, S_(stream), g, ncnt, cells, cell_of_id);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_slice_counts(const DGeom& g, const uint32_t* ncnt, unsigned long long* counts, void* stream) {
  hipLaunchKernelGGL(slice_counts_kernel, dim3(g.S), dim3(WG), 0, S_(stream), g, ncnt, counts);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mdk
