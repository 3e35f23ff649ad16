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
int launch_reduce_state(const DevCase<L, St>& c, hipStream_t s);
template <class L, class St, bool COUPLED>
int launch_set_state(const DevCase<L, St>& c, const double* g, const double* f, const double* J, long t,
                     hipStream_t s);
template <class L, class St, bool COUPLED>
int launch_get_state(const DevCase<L, St>& c, double* g, double* f, double* J, hipStream_t s);
template <class L, class St>
int launch_finalize(const DevCase<L, St>& c, hipStream_t s);
template <class St>
int launch_step3d(const DevCase<D3Q19, St>& c, const Tile& tile, int reduce, hipStream_t s);

// number of workgroups the fused step launches for a case of this shape
inline long fused_blocks(int dim, int nx, int ny, int nz, const Tile& t) {
  if (dim == 2) return long((nx + t.bx - 1) / t.bx) * ((ny + t.ty - 1) / t.ty);
  return long((nx + t.bx - 1) / t.bx) * ((ny + t.by3 - 1) / t.by3) * ((nz + t.ty - 1) / t.ty);
}

}  // namespace vclb
