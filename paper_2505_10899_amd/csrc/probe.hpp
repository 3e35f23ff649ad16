// Host-side launcher of the achievable-bandwidth probe (implemented in probe.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace vclb {

// mode 0 copies n16 16-byte vectors src -> dst, 1 reads src (dst: a 4-byte sink), 2 fills
// dst; `blocks` workgroups of 256 lanes, each lane with `unroll` (1, 2, 4 or 8) vectors in
// flight, non-temporal accesses if `nontemporal`.  Returns -1 for another unroll.
int launch_probe(int mode, int unroll, int nontemporal, void* dst, const void* src, long n16, int blocks,
                 hipStream_t s);

}  // namespace vclb
