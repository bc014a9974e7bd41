// The monitor chain in one pass: SOS cascade, STA/LTA characteristic and the
// two-threshold trigger over one window of a chunk (the energy-detector
// monitor of Section 3.4: a chunk of data in, time-channel events out).
//
// The forward kernel body runs as in filark_sos_stalta_process, y and cf
// written only where the caller asks for them; pass B leaves the window's cf
// in the registers that held y, and the trigger body of trig.hip runs on
// them, so cf need not make a round trip through memory and there is one
// launch per window instead of two.  Outputs, states and events are those of
// the two calls (events as a set; their order in the list depends on timing
// in both).
#include "fwd_body.h"

namespace filark {

namespace fwdk {
namespace {

template <int K, bool WRITE_Y, bool UNIT, bool NT>
__global__ void __launch_bounds__(kMaxWaves * kWave) __attribute__((amdgpu_waves_per_eu(K <= 4 ? 4 : 3)))
mon_kernel(MonParams) {
  const PSrc ps{(kparams_t)dev::kparams<MonParams>()};  // the forward's parameters come first
  const int g = group_of(ps.get()->per_xcd, ps.get()->order);
  if (g >= ps.get()->n_grp) return;  // whole workgroup, before any barrier
  fwd_body<K, 48, true, WRITE_Y, UNIT, false, NT, true>(ps, g);
}

template <int K, bool Y, bool U>
hipError_t launch_m(const MonParams &p, hipStream_t stream) {
  const size_t lds = fwd_lds_bytes(K, p.f.nw, p.f.n_lev, 1 << p.f.cw_log2);
  const dim3 grid((unsigned)fwd_grid(p.f)), block((unsigned)(p.f.nw * kWave));
  if (p.f.nt)
    hipLaunchKernelGGL((mon_kernel<K, Y, U, true>), grid, block, lds, stream, p);
  else
    hipLaunchKernelGGL((mon_kernel<K, Y, U, false>), grid, block, lds, stream, p);
  return hipGetLastError();
}

template <int K>
hipError_t launch_mk(const MonParams &p, bool write_y, bool unit, hipStream_t stream) {
  if constexpr (K >= 2) {
    if (unit) return write_y ? launch_m<K, true, true>(p, stream) : launch_m<K, false, true>(p, stream);
  }
  return write_y ? launch_m<K, true, false>(p, stream) : launch_m<K, false, false>(p, stream);
}

}  // namespace
}  // namespace fwdk

hipError_t launch_monitor(const MonParams &p, int K, bool write_y, bool unit, hipStream_t stream) {
  if (p.f.nw < 1 || p.f.nw > kMaxWaves || p.f.n_t < 1 || p.t.n_t != p.f.n_t || p.t.nw != p.f.nw ||
      p.t.cw_log2 != p.f.cw_log2 || p.t.cap < 0 || !p.t.count || !p.f.sl)
    return hipErrorInvalidValue;
  switch (K) {
    case 1: return fwdk::launch_mk<1>(p, write_y, unit, stream);
    case 2: return fwdk::launch_mk<2>(p, write_y, unit, stream);
    case 3: return fwdk::launch_mk<3>(p, write_y, unit, stream);
    case 4: return fwdk::launch_mk<4>(p, write_y, unit, stream);
    case 5: return fwdk::launch_mk<5>(p, write_y, unit, stream);
    case 6: return fwdk::launch_mk<6>(p, write_y, unit, stream);
    case 7: return fwdk::launch_mk<7>(p, write_y, unit, stream);
    case 8: return fwdk::launch_mk<8>(p, write_y, unit, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace filark
