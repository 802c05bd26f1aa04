// Host-side helpers shared by the single-lattice and the batch C ABI of liblbm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.hpp"

namespace lbm {

// Records the message of a failing call for lbm_last_error() and returns `code`.
lbm_status fail(lbm_status code, const char* fmt, ...);

// Cleanup paths ignore HIP errors on purpose: there is nothing left to report them to.
inline void ignore(hipError_t) {}

#define LBM_HIP_TRY(expr)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return ::lbm::fail(LBM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

struct DeviceGuard {
    int prev = 0;
    int dev = 0;
    explicit DeviceGuard(int d) : dev(d)
    {
        ignore(hipGetDevice(&prev));
        if (prev != dev) ignore(hipSetDevice(dev));
    }
    ~DeviceGuard()
    {
        if (prev != dev) ignore(hipSetDevice(prev));
    }
};

// Derived global parameters of the prescription (Sec. III.B, Sec. IV).
struct Globals {
    double tau_s = 0, tau_q = 0, L1 = 0, L2 = 0, E = 0, E_max = 0;
};

// One validated lattice, ready for upload: flag bytes, links sorted by (site, direction) with the
// caller's index of each, and the per-64-site chunk link offsets.
struct Prepared {
    lbm_params p{};
    Globals g;
    uint32_t nx = 0, ny = 0, n = 0, nchunks = 0;
    int64_t n_fluid = 0, n_links = 0;
    std::vector<uint8_t> flags;
    std::vector<int32_t> chunk;  // nchunks + 1, local link indices
    std::vector<int64_t> order;  // sorted position -> caller's link index
    std::vector<double> q, ubx, uby;
    std::vector<int32_t> dir;
};

// Global parameters of the prescription (Sec. III.B, Sec. IV) from the problem statement; LBM_E_PARAM
// if a relaxation time is not above 1/2.
lbm_status derive_globals(const lbm_params& p, Globals& g);

// Mode ranges, rho0 and the body force of *p, then derive_globals.
lbm_status check_params(const lbm_params& p, Globals& g);

// Validates the problem statement (see lbm_create in include/lbm.h) without touching the device.
lbm_status prepare(const lbm_params* p, const uint8_t* solid, const lbm_link* links, int64_t n_links,
                   Prepared& out);

// Uploads the sorted link inputs of `pr`, runs the fp64 per-link precompute into rows of
// coef64 (row stride `stride`, first link at coef64 + link_off) and, if coef32 is given, its fp32
// copies (same stride and offset); checks 1 + l > 0 and 0 <= r <= 1 and counts clamped and
// non-convex links.  Synchronises `stream`.
lbm_status precompute_links(const Prepared& pr, double* coef64, float* coef32, int64_t stride, int64_t link_off,
                            hipStream_t stream, int32_t& n_clamped, int32_t& n_nonconvex);

// Physical constants of the step kernel in the storage precision.
template <typename T>
Phys<T> make_phys(const lbm_params& p, const Globals& g)
{
    const double s_e = 1.0 / p.tau_e, s_eps = 1.0 / p.tau_eps, s_q = 1.0 / g.tau_q, s_s = 1.0 / g.tau_s;
    Phys<T> ph;
    ph.rho0 = T(p.rho0);
    ph.ax = T(p.ax);
    ph.ay = T(p.ay);
    ph.s_e = T(s_e);
    ph.s_eps = T(s_eps);
    ph.s_q = T(s_q);
    ph.s_s = T(s_s);
    ph.c_e = T(1.0 - 0.5 * s_e);
    ph.c_eps = T(1.0 - 0.5 * s_eps);
    ph.c_q = T(1.0 - 0.5 * s_q);
    ph.c_s = T(1.0 - 0.5 * s_s);
    return ph;
}

// LDS a step-kernel block may use for its link staging area.
constexpr size_t kMaxLds = 64 * 1024;

}  // namespace lbm
