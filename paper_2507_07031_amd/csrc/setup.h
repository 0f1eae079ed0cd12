// Internal interface of the Lagrange-basis setup kernel (msm.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field.h"
#include "msm.h"

namespace zk {

// Lagrange basis of H = <omega_(2^L)>: out[j] = [l_j(tau)] G, j < 2^L, with
//   l_j(tau) = c omega^j / (tau - omega^j),  c = (tau^n - 1) / n   (tau not in H),
//   l_j(tau) = [tau == omega^j]                                     (tau in H).
// c_mont: c in Montgomery form (ignored when tau_in_h); tw_lo / tw_hi: the
// split tables of omega_(2^28)^e.  gtab_dev as for srs_from_tau.
hipError_t srs_lagrange_from_tau(Tau8 tau, uint32_t L, f29 c_mont, bool tau_in_h, const f29* tw_lo,
                                 const f29* tw_hi, uint32_t* out, uint32_t* gtab_dev, hipStream_t s);

}  // namespace zk
