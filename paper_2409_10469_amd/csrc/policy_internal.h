// Library-internal helpers shared by the controller and the proposal network.
#pragma once
#include <hip/hip_runtime.h>

#include "mppi.h"

struct mppi_policy;

namespace mppi_host {
// features of state d_x (37) and d_cmd_origin (cmd[3], origin[2]) -> forward pass of one
// row -> proposal centre and std for nk knots per joint, all on stream st
mppi_status policy_infer(mppi_policy* p, const float* d_x, const float* d_cmd_origin, int nk, float sigma_max,
                         float* d_center, float* d_sd, hipStream_t st);
const char* policy_error(const mppi_policy* p);
// output rows (B x 144) of raw feature rows (B x 40), B <= max_batch, on stream st
mppi_status policy_forward_rows(mppi_policy* p, const float* d_in, int B, float* d_out, hipStream_t st);
// the bound workspace (null when unbound): a graph that captured the policy's launches
// is stale once it changes
const void* policy_workspace(const mppi_policy* p);
// device pointers of the output standardisation: mean and std of the 72 knot means
mppi_status policy_out_norm(mppi_policy* p, const float** omean, const float** ostd);
// the head's knot-resampling matrices for every knot count, rtab[nk][i][k] (9 x 8 x 6)
void policy_resample_table(float* rtab);
// value at t of the not-a-knot spline through nk knots on [0, T] with knot k = 1, others 0
double spline_basis_at(int nk, double T, int k, double t);
// one plain control step of an unbound controller with its workspace in a given device
// region (the static scratch of mppi_step_static); see mppi_api.cpp
mppi_status step_in_region(mppi_ctx* c, void* region, size_t bytes, const float* d_x0, float* d_nominal,
                           float* d_u0_out, hipStream_t st);
}  // namespace mppi_host
