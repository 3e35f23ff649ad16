// Host-side interface of the label reductions (reduce.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <stddef.h>

#include "vclb.h"

namespace vclb {

using LabelObs = vclb_obs;

// Each workgroup of the label reduction owns a chunk of at least kLabelChunkMin nodes;
// at most kLabelMaxBlocks workgroups.
constexpr long kLabelChunkMin = 2048;
constexpr int kLabelMaxBlocks = 512;

int label_blocks(long n);
// device bytes of scratch one label reduction of n nodes into nlabels labels needs
size_t label_scratch_bytes(long n, int nlabels);

// phi: N values of the order parameter (device); labels: N int32 (device).  Writes
// nlabels vclb_obs records followed by one double (the number of nodes whose label is
// >= nlabels) at scratch + the partials' aligned size; see label_result.
template <class R>
int launch_label_reduce(const R* phi, const int* labels, long n, int nx, int ny, int nlabels, long step,
                        void* scratch, hipStream_t s);

// where launch_label_reduce leaves its results inside scratch
inline size_t label_result_offset(long n, int nlabels) {
  const size_t nb = size_t(label_blocks(n));
  const size_t part = (size_t(nlabels) * 13 + 1) * nb * sizeof(double);
  return ((part + 255) / 256) * 256;
}

// Fixed device scratch for callers that cannot allocate (vclb_reduce_static): one array
// of kStaticScratchBytes per device, its device address looked up once per device.
constexpr size_t kStaticScratchBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;
// the scratch array's device address on the current device (0) or a HIP error (-3) / a
// device index beyond kMaxDevices (-1)
int static_scratch(void** ptr);

}  // namespace vclb
