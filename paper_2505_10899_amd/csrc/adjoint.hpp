// Buffers and launchers of the FP64 D2Q9 adjoint (adjoint.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "devcase.hpp"

namespace vclb {

constexpr int kSeedFields = 10;   // per label: sum, d[3], dd[6] (xx, yy, zz, xy, xz, yz)

// Device buffers of one backward sweep, each N-major ([component][node]).
struct AdjArgs {
  const double* lg_in;    // [9][N] lg of step t + 1
  const double* lf_in;    // [9][N]
  const double* lJ_in;    // [2][N]
  double* lg_out;         // [9][N] lg of step t
  double* lf_out;         // [9][N]
  double* lJ_out;         // [2][N]
  double* lphi;           // [N] adjoint of phi: read for t + 1 by k_adj_local, then rewritten for t
  double* aux;            // [6][N] stencil-input adjoints of the current step
  double* param_part;     // [2][workgroups] running (dJ/dsigma, dJ/dM) per workgroup
  const double* seed;     // [labels][kSeedFields] device copy of the moment weights
  double beta4_per_sigma;   // 4 beta / sigma = 48 / W
  double kappa_per_sigma;   // kappa / sigma = 3 W / 2
  unsigned mobility_rows;   // bit k: s_k^g is the default 1 / tau_g
  double normal_tau2;       // n is held fixed (no derivative) where |grad psi|^2 < normal_tau2
};

long adj_blocks(long n);
int launch_adj_zero(double* p, long count, hipStream_t s);
int launch_adj_seed(const DevCase<D2Q9, StoreF64>& c, const AdjArgs& a, hipStream_t s);
int launch_adj_step(const DevCase<D2Q9, StoreF64>& c, const AdjArgs& a, hipStream_t s);
int launch_adj_init(const DevCase<D2Q9, StoreF64>& c, const AdjArgs& a, const double* phi0, const double* u0,
                    double* dphi0, hipStream_t s);
int launch_adj_params(const AdjArgs& a, int nblocks, double* out, hipStream_t s);

}  // namespace vclb
