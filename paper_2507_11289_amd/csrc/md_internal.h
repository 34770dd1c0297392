// md_internal.h -- types shared by the device kernels and the host runtime of libmd.
//
// Data layout in HBM (one simulation or one served run):
//   two cell buffers (parity 0/1).  A cell owns CELL_CAP atom slots stored as one
//   block: x[64] y[64] z[64] vx[64] vy[64] vz[64] (FP64), id[64] (u32), then
//   r[64] (FP32 x, y, z, 0): the position relative to the cell's corner, x - gx l rounded
//   once (the FP32 pair path stages these: one 16-byte load per atom, two cache lines for
//   16 atoms instead of three).
//   Cells are numbered slice-major: cell = slice * cells_per_slice +
//   ((gx mod ncx) * Gy + gy) * Gz + gz, so a slice is one contiguous range of blocks.
//   ncnt[p][cell]: atoms in the cell; nin[p][cell]: atoms that moved in from
//   another cell during the last step (appended from the top slot downwards).
//   Within a finalised cell, atoms are ordered by id.
#pragma once
#include <stdint.h>

namespace mdk {

constexpr int CELL_CAP = 64;                 // slots per cell (one wavefront)
constexpr int CELL_DOUBLES = 6 * CELL_CAP;   // x y z vx vy vz
constexpr int CELL_BYTES = CELL_DOUBLES * 8 + CELL_CAP * 4 + CELL_CAP * 16;  // 4352 = 17 x 256
constexpr int WG = 256;                      // threads per workgroup (4 waves)
constexpr int WAVES = WG / 64;
constexpr int BLOCK_CELLS = WAVES;            // cells of one z-column per staged block (one per wave)
constexpr int MAX_XQ = 8;                    // work queues at most: one per XCD (L2 domain)
constexpr int XQ_STRIDE = 32;                // queue counters 256 bytes apart

// error word bits
constexpr uint32_t ERR_NONFINITE = 1u;
constexpr uint32_t ERR_DISPLACEMENT = 2u;
constexpr uint32_t ERR_CAPACITY = 4u;
constexpr uint32_t ERR_WATCHDOG = 8u;
constexpr uint32_t ERR_BADINPUT = 16u;
constexpr uint32_t ERR_INJECTED = 32u;

struct DGeom {
  double L[3];
  double halfL[3];
  double l[3];
  double inv_l[3];
  double inv_ncx, inv_cps, inv_G[3];  // 1/ncx, 1/cps, 1/G rounded to FP64: exact quotients
                                      // of non-negative ints (see qdiv)
  double rc2;      // rc^2
  double uc;       // pair energy at rc (subtracted from every pair energy)
  double dt, hdt;  // step and half step
  float rc2_f;     // rc^2 in FP32
  float rc2_lo_f;  // FP32 pairs with r2 <= rc2_lo_f are in range for certain
  float rc2_hi_f;  // FP32 pairs with r2 >  rc2_hi_f are out of range for certain
  float rc2_pre_f; // pre-filter threshold: every pair with FP32 r2 <= rc2_hi_f has a matrix-core
                   // estimate of r2 below it
  float uc_f;
  int S;           // slices
  int ncx;         // cell layers per slice
  int G[3];        // cells per axis
  int cps;         // cells per slice
  int ncell;       // cells in total
  int prec;        // 0 FP64, 1 FP32 force
  int cap;         // atoms a cell may hold (at most CELL_CAP; lower to force capacity errors)
};

struct RunArgs {
  DGeom g;
  unsigned char* cells[2];
  uint32_t* ncnt[2];
  uint32_t* nin[2];
  uint32_t* cntA;               // per slice: finalise items completed in this launch (+nchA at start
                                // with a fixed claim order)
  uint32_t* cntF;               // per slice: force/integrate items completed in this launch
  double* epart;                // [nsample][S][nch][3] partial U, K, W (energy steps)
  uint32_t* miglog;             // [nsteps][S][2] or null
  unsigned long long* migcum;   // [S][2] cumulative migrations
  unsigned long long* paircnt;  // [2] candidates, in-range (count mode)
  uint32_t* err;                // error word of this run
  uint32_t* abort;              // set on any error of this run; its waits give up
  const uint32_t* order;        // claim table of one round of wlev steps, 2*S*wlev entries:
                                // (j << 16) | (phase << 15) | slice, j = step within the round
  int wlev;                     // steps per round of a fixed claim order (1, or the wavefront's
                                // time levels)
  long long t0;                 // absolute step at the start of the launch
  int nsteps;                   // steps in this launch
  int par0;                     // parity of the sorted buffer at t0
  int first;                    // 1: stored velocities are v(t0) (not half-step velocities)
  int nch;                      // force (and thermostat integrate) items per slice and step
  int nchA;                     // finalise items per slice and step (fewer than nch with the
                                // dataflow scheduler: they are short, and every item pays a
                                // release and an acquire)
  int every;                    // energy sampling interval (0 = none)
  int count;                    // count candidates / in-range partners
  long long fail_at;            // debug fault injection step (-1 off)
  int ips;                      // items per step: S * (nch + nchA) (+ S * nch with the thermostat)
  double thermo_T;              // velocity-scaling thermostat target temperature (0: off)
  double* fbuf;                 // thermostat: F(t) per slot of the step's cells [ncell][3][64]
  double* kpart;                // thermostat: [S][nch][2] kinetic energy and atoms of v(t)
  uint32_t* cntK;               // thermostat: per slice, force items completed in this launch
  // XCD work queues (LaunchArgs::nq > 1): queue x holds the items of slices
  // [xfirst[x], xfirst[x + 1]) and its first-step force items start at slot q0[x]
  int xfirst[MAX_XQ + 1];
  long long q0[MAX_XQ];
};

struct TraceRec {
  uint32_t k, slice, chunk, phase;
  uint32_t hw_id, launch;
  uint32_t xcd, queue;
  unsigned long long t_claim, t_ready, t_done;
};

struct LaunchArgs {
  RunArgs* runs;
  int nruns;
  int nrounds;
  const long long* round_base;  // [nrounds + 1] first ticket of each round
  const int* round_active;      // [nrounds] runs active in the round (runs sorted by steps)
  const long long* run_prefix;  // [nruns + 1] prefix sums of ips
  unsigned long long* ticket;   // claim counter
  long long watchdog_ticks;     // wall_clock64 ticks a wait may take
  TraceRec* trace;              // one record per ticket, or null
  uint32_t launch_index;
  int mode;                     // 0 dataflow queue, 1 fixed claim order
  unsigned long long* q;        // dataflow: item slots (top bit set once pushed)
  unsigned long long* q_tail;   // dataflow: next free slot of queue x at q_tail[XQ_STRIDE x]
  uint32_t* launch_err;         // dataflow: a queue wait exceeded the watchdog
  long long total;              // items in the launch
  // Dataflow work queues.  nq = 1: one queue for the device, every item synchronises at
  // agent scope.  nq > 1: one queue per XCD; queue x occupies slots [qoff[x], qoff[x+1])
  // of q, holds the items of each run's slices [xfirst[x], xfirst[x+1]) and is served by
  // the workgroups running on XCD x only, so items whose inputs all come from the same XCD
  // exchange data through that XCD's L2 (see release_full).  The claim counter of queue x
  // is ticket[XQ_STRIDE x].
  int nq;
  long long qoff[MAX_XQ + 1];
  long long prefill[MAX_XQ];    // first-step force items of all runs in queue x
};

// Host-callable launch wrappers (defined in md_device.hip).
int launch_clear_u32(uint32_t* p, long long n, uint32_t value, void* stream);
int launch_load_scatter(const DGeom& g, const double* pos, const double* vel, long long n,
                        unsigned char* cells, uint32_t* ncnt, uint32_t* err, void* stream);
int launch_sort_cells(const DGeom& g, unsigned char* cells, uint32_t* ncnt, uint32_t* err,
                      void* stream);
int launch_init(const LaunchArgs& la, long long work, void* stream);
int launch_gather_errors(const RunArgs* runs, int nruns, uint32_t* out, void* stream);
// kind: 0 plain steps, 1 energy-sampled steps, 2 pair counting (see the kernels)
int persistent_grid(int prec, int kind, int nvt, int* blocks_per_cu, int* cus);
int launch_persistent(const LaunchArgs& la, int prec, int kind, int nvt, int grid, void* stream);
int launch_sync(const DGeom& g, const unsigned char* cells, const uint32_t* ncnt, int first,
                double* out_pos, double* out_vel, double* out_force, double* epart,
                uint32_t* err, void* stream);
int launch_cells_of(const DGeom& g, const uint32_t* ncnt, const unsigned char* cells,
                    long long* cell_of_id, void* stream);
int launch_slice_counts(const DGeom& g, const uint32_t* ncnt, unsigned long long* counts,
                        void* stream);
int sync_blocks(const DGeom& g);

}  // namespace mdk
