// Internal definitions shared by the host layer (jefi_api.cpp) and the
// kernels (jefi_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/libjefi.h"

namespace jefi {

// Source bricks: 2x2x2 cells, the unit of the ring layout and of staging.
constexpr int kBrickCells = 8;
// Observation tile: 8x8x8 points per workgroup, 4x4x4 per wavefront.
constexpr int kTileEdge = 8;
constexpr int kThreads = 512;
// Slice-window slots staged per source cell and launch variant.
constexpr int kWmax = 32;
// Largest table of slice-boundary thresholds a launch stages in LDS
// (FP32 and FP64 kernels: the FP64 staging planes take twice the LDS).
constexpr int kThrMax = 1024;
constexpr int kThrMax64 = 512;

struct GridD {
  int n[3];
  double o[3];
  double h[3];
};

// Everything a pair-kernel launch needs; passed by value.
// Time-stencil readings (pair kernels): derivative as the slope of the
// linear interpolant; history before the oldest slice held at its values;
// cubic time interpolation through slices k-2 .. k+1; a history that starts
// at the oldest slice (earlier retarded times contribute nothing, stencils
// reaching before it read it).
constexpr int kStencilSlope = 1;
constexpr int kStencilHold = 2;
constexpr int kStencilCubic = 4;
constexpr int kStencilCut = 8;

struct PairParams {
  GridD src, obs;
  int nbx, nby, nbz;
  int n_bricks;
  int ntx, nty, ntz;
  int n_tiles;
  int n_splits;
  int bricks_per_split;
  int n_wg;
  // time axis (logical slice units, oldest used slice = 0)
  int a_i;
  double a_f;
  double inv_cdt;
  double inv_dt;
  int nt;
  int capacity;
  int slot_base;         // (newest - nt + 1) mod capacity
  double screen[3];
  double margin;         // slack on box-derived slice bounds, slice units
  double near_slack;     // slack on the box screening test, length units
  float guard;           // FP32 index guard half-width, slice units
  int use_thr;           // 1: decide guard-band pairs by the r2 threshold table
  int exact_idx;         // 1 (needs use_thr): decide every full-brick pair by the table,
                         // without the FP32 guard test (many pairs near integer positions)
  int thr_lo;            // table covers floor positions thr_lo .. thr_lo + thr_n - 1
  int thr_n;
  double* thr;           // device table of thr_n thresholds (filled by the threshold kernel)
  int tile_z;            // observation tile edge in z: 8 (512 threads) or 4 (256 threads)
  const void* ring;      // device ring, library layout
  unsigned ring_bytes_rs;  // ring bytes when below 2^31 - 16 (buffer-addressed staging), else 0
  long long slot_elems;  // elements (of the ring dtype) per slot
  double* partial;       // FP64 [n_splits][6][n_obs] (unscaled sums)
  void* E;
  void* B;
  int out_f64;
  double pref;           // dOmega / (4 pi)
  unsigned long long* fp;  // fingerprint output [n_obs][4]
  int direct;            // 1: one split, the pair kernel writes E/B itself
  int stencil;           // kStencil* bits, or 0 (interpolated backward differences,
                         // zero history before the oldest slice)
};

struct EpilogueParams {
  const double* partial;
  int n_splits;
  long long n_obs;
  double pref;
  void* E;
  void* B;
  int out_f64;
};

// Batched launch: per-instance parameters and work items live in device memory.
// Instances of a batch fall in up to two launch groups (8x8x8 and 8x8x4
// observation tiles), each a persistent launch over its own range of the
// item list with its own queue head.
struct BatchDevice {
  const PairParams* params;   // [n_inst]
  const int2* items;          // [n_items] (instance, workgroup id within the instance)
  const int* counts;          // counts[0] = n_inst; group g: counts[1 + 2g] = its items,
                              // counts[2 + 2g] = index of its first item
  int* counter;               // work-queue heads, one per group
  const EpilogueParams* epi;  // [n_inst] (n_splits == 0 for instances written directly)
  const long long* epi_prefix;  // [n_inst + 1] cumulative 6 * n_obs of instances with an epilogue
  int group;                  // the group a persistent launch serves
};

struct DumpParams {
  GridD src, obs;
  int a_i;
  double a_f;
  double inv_cdt;
  double screen[3];
  float guard;
  int use_f64;
  int* out;
};

// Launchers (jefi_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_zero(void* p, unsigned long long bytes, hipStream_t s);
hipError_t launch_ingest(const void* slice, void* slot, const GridD& src, int nbx, int nby,
                         int is_f64, hipStream_t s);
// All n_slots slots of a history in host layout [n_slots][4][n_src] (device
// memory) into the first n_slots ring slots.
hipError_t launch_ingest_slots(const void* hist, void* ring, const GridD& src, int nbx, int nby, int n_slots,
                               int is_f64, hipStream_t s);
// wsel: slots staged per cell (32; 64 or 128 for long windows, 8x8x8 tiles
// only, 64 at most in FP64); ignored when multi_chunk.
hipError_t launch_pairs(const PairParams& p, int is_f64, int fingerprint, int multi_chunk, int wsel,
                        hipStream_t s);
hipError_t launch_thresholds(double* out, int lo, int n, double af, double icdt, hipStream_t s);
// Kernel entry points of a batched evaluation, for graph nodes.
void* batch_reset_kernel();
void* batch_threshold_kernel();
// idx: index mode of the FP32 kernel (1 = threshold table for every pair,
// needs use_thr in every instance; 0 = guard band).
void* batch_pair_kernel(int is_f64, int wz, int idx, int stg);  // stg: bit 0 cubic, bit 1 history start
void* batch_epilogue_kernel();
int batch_pair_threads(int wz);
hipError_t launch_epilogue(const EpilogueParams& p, hipStream_t s);
hipError_t launch_fill_zero_fields(void* E, void* B, long long n_obs, int out_f64, hipStream_t s);
hipError_t launch_dump(const DumpParams& p, hipStream_t s);

// The library's error state (jefi_last_error, the sticky device failure),
// for the parts of the library outside jefi_api.cpp.
jefi_status report_error(jefi_status st, const char* msg);
jefi_status report_hip(hipError_t e, const char* what);  // sticky: every later call fails
bool device_failed();

// Compute units of the current device.
int device_cus();
// A non-blocking stream whose kernels run only on compute units
// first_cu .. first_cu + n_cus - 1 (a CU mask); false if the device or
// runtime refuses the mask (no stream is created then).
bool create_stream_on_cus(hipStream_t* s, int first_cu, int n_cus);
// jefi_eval_batch whose persistent launches fill the workgroup slots of
// grid_cus compute units (any count from 1 to the device's), for callers
// that run the batch on a stream restricted to that many units.
jefi_status eval_batch_on_cus(const jefi_problem* probs, int32_t n, const jefi_options* opt, void* stream,
                              int grid_cus);

// Fixed device scratch of the allocation-free evaluation (per GPU): the
// threshold table and FP64 split partials.
constexpr unsigned long long kNoAllocScratchBytes = 128ull << 20;
// Address of the current device's copy (looked up on its first use).
hipError_t noalloc_scratch(void** out);

}  // namespace jefi
