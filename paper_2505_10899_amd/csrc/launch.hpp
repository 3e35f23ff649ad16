// Host-side launcher declarations (implemented next to their kernels).
#pragma once
#include <hip/hip_runtime.h>

#include "devcase.hpp"

namespace vclb {

// Launch shape of the fused step: bx lanes (x columns) per workgroup marching over ty
// rows; for D3Q19 the workgroup covers by3 rows of y and marches over ty planes of z.
struct Tile {
  int bx = 256;
  int ty = 32;
  int by3 = 4;
};

template <class L, class St, bool COUPLED>
int launch_init(const DevCase<L, St>& c, const double* phi0, const double* u0, hipStream_t s);
template <class L, class St, bool COUPLED>
int launch_step_plain(const DevCase<L, St>& c, int reduce, hipStream_t s);
template <class L, class St, bool COUPLED>
int launch_step_fused(const DevCase<L, St>& c, const Tile& tile, int reduce, hipStream_t s);
template <class L, class St, bool COUPLED>
int launch_observe(const DevCase<L, St>& c, unsigned mask, double* out, hipStream_t s);
template <class L, class St>
int launch_phi_psi(const DevCase<L, St>& c, hipStream_t s);
template <class L, class St>
int launch_reduce_state(const DevCase<L, St>& c, hipStream_t s);
// the global volume correction's reference volume, from the current state
template <class L, class St>
int launch_mass_ref(const DevCase<L, St>& c, hipStream_t s);
template <class L, class St, bool COUPLED>
int launch_set_state(const DevCase<L, St>& c, const double* g, const double* f, const double* J, long t,
                     hipStream_t s);
template <class L, class St, bool COUPLED>
int launch_get_state(const DevCase<L, St>& c, double* g, double* f, double* J, hipStream_t s);
template <class L, class St>
int launch_finalize(const DevCase<L, St>& c, hipStream_t s);
template <class St>
int launch_step3d(const DevCase<D3Q19, St>& c, const Tile& tile, int reduce, hipStream_t s);
template <class St>
size_t step3d_lds_bytes(int bx, int by3);   // LDS of the fused 3D step for a bx x by3 section

struct BatchArgs {
  const int4* items;        // (case, x0, y0, y1) of every work item, case-major; x0 < 0: a
                            // flattened band of rows [y0, y1), else a strip of columns from x0
  int nitems;
  const int2* runs;         // (first item, item count) of each resident workgroup slot
  const int2* case_items;   // (first item, item count) per case
  int ncases;
  double* part_w;           // [12][nitems] partials written by this launch
  const double* part_r;     // [12][nitems] partials of the previous launch
  int pend;                 // part_r holds partials of step pend_step still to be summed
  long pend_step;
  long t;                   // step index of the state this launch reads
  int reduce;               // record the reductions of this step
  int cap;                  // LDS ring entries of the flattened march (power of two)
  int lag;                  // its lag in chunks (1 or 3)
  int unit;                 // every case has unit rates outside the g flux and f stress rows
  int visc;                 // some case has unequal viscosities (per-node tau_f)
  unsigned* ticks;          // if set: per run slot, the wall-clock ticks its workgroup spent
                            // on its run (balancing launches only)
};

template <class St>
int launch_batch_step(const void* cases, const BatchArgs& a, int blocks, int bx, hipStream_t s);
template <class St>
size_t batch_lds_bytes(int cap, int bx);
template <class St>
int launch_batch_fold(const void* cases, const BatchArgs& a, hipStream_t s);
template <class St>
int batch_max_blocks_per_cu(int bx, int cap, int lag, bool unit, bool visc);

// Entries per plane of the populations and of J for a case of n nodes: n rounded up to a
// multiple of 64, so that every plane starts on a cache line.
inline long plane_stride(long n) { return (n + 63) / 64 * 64; }

// Lag (in chunks of B lanes) of the flattened batched march for rows of nx nodes: the
// update of stored node e needs phi up to node e + nx + 1, so lag B >= nx + 1; 1 or 3 (the
// register FIFO holds lag + 1 chunks), 0 if the rows are too wide for B lanes.
inline int flat_lag(int nx, int B) {
  const int need = (nx + 1 + B - 1) / B;
  return need <= 1 ? 1 : (need <= 3 ? 3 : 0);
}

// LDS ring entries (a power of two) of the flattened march.  The oldest stencil input
// read in iteration i lies at most P + nx ring positions before chunk i - lag (a row's
// last node reads column 0 of the row above), and the newest entry written in iteration
// i + 1 ends chunk i + 1: (lag + 2) B stored nodes further on, plus two ring positions
// (the padding columns) per row they cross.
inline int flat_ring_cap(int nx, int B, int lag) {
  const long span = long(lag + 2) * B;
  const long need = span + 2 * (span / nx + 1) + 2 * nx + 3;
  int cap = 1;
  while (cap <= need) cap <<= 1;
  return cap;
}

// number of workgroups the fused step launches for a case of this shape
inline long fused_blocks(int dim, int nx, int ny, int nz, const Tile& t) {
  if (dim == 2) return long((nx + t.bx - 1) / t.bx) * ((ny + t.ty - 1) / t.ty);
  return long((nx + t.bx - 1) / t.bx) * ((ny + t.by3 - 1) / t.by3) * ((nz + t.ty - 1) / t.ty);
}

}  // namespace vclb
