// Host-side launch interface of the proposal-step helper kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace prop {
// e (Kp x D, sample-major) holds standard Gaussian noise on entry; on exit row 0 is 0,
// row 1 is nominal - center and row n >= 2 is sd * e_n
hipError_t launch_proposal_noise(int Kp, int D, float* e, const float* center, const float* sd, const float* nominal,
                                 hipStream_t st);
// state x (37 floats) and cmd_origin = (cmd[3], origin[2]) -> 40 raw features
hipError_t launch_features(const float* x, const float* cmd_origin, float* feat, hipStream_t st);
}  // namespace prop
