// Forward kernels with 32-row blocks (every section count, fused and
// standalone variants); the kernel body is in fwd_body.h.
#include "fwd_body.h"

namespace filark {

hipError_t launch_fwd_l32(const FwdParams &p, int K, bool stalta, bool write_y, bool unit, bool rev,
                          hipStream_t stream) {
  return fwdk::launch_l<32>(p, K, stalta, write_y, unit, rev, stream);
}

}  // namespace filark
