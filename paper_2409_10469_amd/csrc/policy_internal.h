// Library-internal helpers shared by the controller and the proposal network.
#pragma once
#include <hip/hip_runtime.h>

#include "mppi.h"

struct mppi_policy;

namespace mppi_host {
const char* policy_error(const mppi_policy* p);
// value at t of the not-a-knot spline through nk knots on [0, T] with knot k = 1, others 0
double spline_basis_at(int nk, double T, int k, double t);
}  // namespace mppi_host
