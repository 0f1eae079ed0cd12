// Device-side input checks (validate.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zk {

constexpr uint32_t VALIDATE_FR = 1u;  // an Fr input was >= r
constexpr uint32_t VALIDATE_G1 = 2u;  // a G1 input was not a canonical point on the curve
constexpr uint32_t VALIDATE_G2 = 4u;  // a G2 input was not a canonical point of order r on the twist

// OR VALIDATE_FR into *flag if any of the n elements (8 words each) is >= r.
hipError_t validate_fr(const uint32_t* v, uint64_t n, uint32_t* flag, hipStream_t s);
// OR VALIDATE_G1 into *flag if any of the n affine points (16 words each) is
// neither (0, 0) nor a canonical point on y^2 = x^3 + 3.
hipError_t validate_g1(const uint32_t* pts, uint64_t n, uint32_t* flag, hipStream_t s);
// OR VALIDATE_G2 into *flag if any of the n G2 points (32 words each) is
// neither all zeros nor a canonical point of order r on the twist.
hipError_t validate_g2(const uint32_t* pts, uint64_t n, uint32_t* flag, hipStream_t s);

}  // namespace zk
