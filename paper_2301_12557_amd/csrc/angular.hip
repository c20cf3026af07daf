// angular.hip -- angular pair counts.  The method applies to pairs of points
// on the sky directly (Sect. 3.1; angular statistics are the future work of
// Sect. 6): a sky position is a unit vector, and the angle theta between two
// of them maps one to one onto their chord 2 sin(theta / 2), so angular bins
// are chord bins of the unit vectors.  Counting then runs through the s path
// unchanged, in an open box around the unit sphere.
#include <math.h>

#include <vector>

#include "internal.h"

namespace fcfc {

// (cos dec cos ra, cos dec sin ra, sin dec), angles in degrees
__global__ void k_radec_to_unit(const double* __restrict__ ra, const double* __restrict__ dec, int64_t n,
                                double* __restrict__ xyz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = ra[i] * (M_PI / 180.0);
    const double d = dec[i] * (M_PI / 180.0);
    double sa, ca, sd, cd;
    sincos(a, &sa, &ca);
    sincos(d, &sd, &cd);
    xyz[3 * i] = cd * ca;
    xyz[3 * i + 1] = cd * sa;
    xyz[3 * i + 2] = sd;
}

}  // namespace fcfc

using namespace fcfc;

extern "C" fcfc_status fcfc_radec_to_unit(const double* d_ra_deg, const double* d_dec_deg, int64_t n, double* d_xyz,
                                          void* stream) {
    clear_error();
    if (n < 0 || (n > 0 && (!d_ra_deg || !d_dec_deg || !d_xyz))) {
        set_error("radec_to_unit: null arrays or negative size");
        return FCFC_EINVAL;
    }
    if (n == 0) return FCFC_OK;
    hipLaunchKernelGGL(k_radec_to_unit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       d_ra_deg, d_dec_deg, n, d_xyz);
    FCFC_HIP(hipGetLastError());
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_angular_plan(const double* theta_deg, int32_t n, const fcfc_tuning* tune,
                                         double* chord_out, fcfc_plan_t* out) {
    clear_error();
    if (!theta_deg || n < 1 || !out) {
        set_error("angular_plan: need at least one bin and an output");
        return FCFC_EINVAL;
    }
    std::vector<double> c((size_t)n + 1);
    for (int k = 0; k <= n; k++) {
        const double t = theta_deg[k];
        if (!(t >= 0.0 && t <= 180.0)) {
            set_error("angular_plan: angular edge %d = %g outside [0, 180] degrees", k, t);
            return FCFC_EEDGES;
        }
        c[k] = 2.0 * sin((t * (M_PI / 180.0)) / 2.0);
    }
    fcfc_plan_t p = nullptr;
    FCFC_TRY(fcfc_plan_create(FCFC_BIN_S, FCFC_LOS_Z, c.data(), n, nullptr, 0, 0.0, tune, &p));
    // unit vectors lie in [-1, 1]^3 (the margin covers their rounding)
    const double lo[3] = {-1.0 - 1e-9, -1.0 - 1e-9, -1.0 - 1e-9};
    const double hi[3] = {1.0 + 1e-9, 1.0 + 1e-9, 1.0 + 1e-9};
    fcfc_status s = fcfc_plan_set_bounds(p, lo, hi);
    if (s != FCFC_OK) {
        fcfc_plan_free(p);
        return s;
    }
    if (chord_out)
        for (int k = 0; k <= n; k++) chord_out[k] = c[k];
    *out = p;
    return FCFC_OK;
}
