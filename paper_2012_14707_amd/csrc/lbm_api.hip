// Host side of liblbm: the C ABI declared in include/lbm.h.
//
// lbm_create validates the problem statement (mask and wall-link table of Sec. III.A), derives
// the global parameters of the prescription (Sec. III.B) on the host in fp64, uploads the mask as
// one flag byte per site and the links sorted by (site, direction), and runs the per-link fp64
// precompute on the device.  lbm_step then launches only the fused step kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.hpp"

namespace {

thread_local std::string g_last_error;

lbm_status fail(lbm_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail(LBM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

constexpr double kPi = 3.14159265358979323846;

const int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

bool is_set(double v) { return std::isfinite(v) && v > 0.0; }

// LDS a step-kernel block may use for its link staging area.
constexpr size_t kMaxLds = 64 * 1024;

}  // namespace

struct lbm_ctx {
    lbm_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t nx = 0, ny = 0, n = 0;
    uint32_t ps = 0;  // population plane stride: n rounded up to whole 64-site chunks
    int64_t n_fluid = 0, n_links = 0;
    double tau_s = 0, tau_q = 0, L1 = 0, L2 = 0, E = 0, E_max = 0;
    int32_t n_clamped = 0, n_nonconvex = 0;
    std::vector<int64_t> order;  // sorted position -> caller's link index
    uint8_t* d_flags = nullptr;
    int32_t* d_chunk = nullptr;
    double* d_coef64 = nullptr;  // 8 rows of n_links
    float* d_coef32 = nullptr;   // 5 rows of n_links (fp32 storage only)
    void* d_buf[2] = {nullptr, nullptr};   // population planes, two time levels
    void* d_link[2] = {nullptr, nullptr};  // per-link incoming populations, two time levels
    int cur = 0;
    std::vector<int32_t> chunk;            // host copy of the chunk link offsets
    uint32_t nchunks = 0;
    uint32_t lds_links = 0;                // LDS link slots for the current block size
    double* d_uprev = nullptr;   // 2 n
    double* d_partial = nullptr;
    double* d_result = nullptr;  // 4
    double* h_result = nullptr;  // pinned, 4
    double* d_stage = nullptr;   // 3 n, for host-side moments and fields
    int64_t steps = 0;
    bool uprev_valid = false;
    int block = 256;
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool have_timing = false;
    int64_t timed_steps = 0;
    bool on_device = false;

    bool fp32() const { return p.precision == LBM_FP32_SHIFTED; }
    size_t pop_bytes() const { return (fp32() ? 4 : 8) * size_t(9) * ps; }
    size_t link_bytes() const { return (fp32() ? 4 : 8) * size_t(n_links > 0 ? n_links : 1); }
    lbm::Geo geo() const { return lbm::Geo{d_flags, d_chunk, n, nx, ny, nchunks, ps}; }
    // Most wall links owned by one block of `blk` sites.
    uint32_t max_links_per_block(int blk) const
    {
        const uint32_t per = uint32_t(blk) / lbm::kChunk;
        uint32_t best = 0;
        for (uint32_t c0 = 0; c0 < nchunks; c0 += per) {
            const uint32_t c1 = std::min(c0 + per, nchunks);
            best = std::max(best, uint32_t(chunk[c1] - chunk[c0]));
        }
        return best;
    }
};

namespace {

// Cleanup paths ignore HIP errors on purpose: there is nothing left to report them to.
inline void ignore(hipError_t) {}

void release(lbm_ctx* c)
{
    if (!c) return;
    if (!c->on_device) {
        delete c;
        return;
    }
    int prev = 0;
    ignore(hipGetDevice(&prev));
    ignore(hipSetDevice(c->device));
    ignore(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    for (void* ptr : {static_cast<void*>(c->d_flags), static_cast<void*>(c->d_chunk), static_cast<void*>(c->d_coef64),
                      static_cast<void*>(c->d_coef32), c->d_buf[0], c->d_buf[1], c->d_link[0], c->d_link[1],
                      static_cast<void*>(c->d_uprev),
                      static_cast<void*>(c->d_partial), static_cast<void*>(c->d_result),
                      static_cast<void*>(c->d_stage)})
        if (ptr) ignore(hipFree(ptr));
    if (c->h_result) ignore(hipHostFree(c->h_result));
    if (c->ev0) ignore(hipEventDestroy(c->ev0));
    if (c->ev1) ignore(hipEventDestroy(c->ev1));
    ignore(hipSetDevice(prev));
    delete c;
}

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

// Global parameters of the prescription, Sec. III.B and Sec. IV.
lbm_status derive_globals(lbm_ctx* c)
{
    const lbm_params& p = c->p;
    const double sq = std::sqrt(6.0 / kPi);
    c->tau_s = is_set(p.tau_s_override) ? p.tau_s_override : 0.5 + sq * p.kn * p.h;  // Eq. (tKnrela)
    if (!(c->tau_s > 0.5)) return fail(LBM_E_PARAM, "tau_s = %g must exceed 1/2", c->tau_s);
    c->L1 = std::isnan(p.L1) ? (2.0 - p.sigma) * (1.0 - 0.1817 * p.sigma) / p.sigma : p.L1;
    c->L2 = std::isnan(p.L2) ? 1.0 / kPi + 0.5 * c->L1 * c->L1 : p.L2;
    if (!std::isfinite(c->L1) || !std::isfinite(c->L2)) return fail(LBM_E_PARAM, "slip coefficients not finite");
    const double ts = c->tau_s, t2 = 2.0 * ts - 1.0;
    // Eq. (EqECond): tau_q > 1/2  <=>  E < E_max
    c->E_max = (kPi * ts * c->L2 - 3.0 * std::sqrt(kPi / 6.0) * c->L1) * t2 / (12.0 * ts) - 0.5;
    c->E = std::isnan(p.E) ? std::min(-0.65, c->E_max - 0.05) : p.E;
    // Eq. (NSliCoertstq)
    c->tau_q = is_set(p.tau_q_override)
                   ? p.tau_q_override
                   : (t2 * (ts * std::sqrt(6.0 * kPi) * c->L2 - c->L1) - 2.0 * sq * ts * (1.0 + 6.0 * c->E)) /
                         (8.0 * sq * ts + 4.0 * c->L1 * t2);
    if (!(c->tau_q > 0.5)) return fail(LBM_E_PARAM, "tau_q = %g must exceed 1/2 (E = %g, bound %g)", c->tau_q, c->E,
                                       c->E_max);
    const double others[4] = {p.tau_rho, p.tau_e, p.tau_eps, p.tau_j};
    for (double t : others)
        if (!(t > 0.5)) return fail(LBM_E_PARAM, "relaxation time %g must exceed 1/2", t);
    return LBM_OK;
}

}  // namespace

extern "C" {

int32_t lbm_version(void) { return 10000; }

const char* lbm_last_error(void) { return g_last_error.c_str(); }

lbm_status lbm_params_default(lbm_params* p)
{
    if (!p) return fail(LBM_E_INVAL, "null params");
    std::memset(p, 0, sizeof *p);
    p->nx = p->ny = 0;
    p->kn = 0.0;
    p->h = 1.0;
    p->sigma = 1.0;
    p->L1 = p->L2 = p->E = std::nan("");
    p->tau_rho = 1.0;
    p->tau_e = 1.1;
    p->tau_eps = 1.2;
    p->tau_j = 1.0;
    p->l_mode = LBM_L_PAPER;
    p->r_mode = LBM_R_FROM_LEFF;
    p->diffuse = LBM_DIFFUSE_NODE;
    p->precision = LBM_FP64;
    p->rho0 = 1.0;
    return LBM_OK;
}

lbm_status lbm_create(const lbm_params* p, const uint8_t* solid, const lbm_link* links, int64_t n_links,
                      void* stream, lbm_ctx** out)
{
    if (!out) return fail(LBM_E_INVAL, "null output pointer");
    *out = nullptr;
    if (!p || !solid || (n_links > 0 && !links) || n_links < 0) return fail(LBM_E_INVAL, "null or negative input");
    if (p->nx <= 0 || p->ny <= 0) return fail(LBM_E_INVAL, "lattice size %d x %d", p->nx, p->ny);
    const uint64_t n64 = uint64_t(p->nx) * uint64_t(p->ny);
    if (n64 >= (uint64_t(1) << 31)) return fail(LBM_E_INVAL, "lattice of %llu sites exceeds 2^31", (unsigned long long)n64);
    if (p->l_mode < 0 || p->l_mode > 7 || p->r_mode < 0 || p->r_mode > 2 || p->diffuse < 0 || p->diffuse > 1 ||
        p->precision < 0 || p->precision > 1)
        return fail(LBM_E_INVAL, "mode out of range");
    if (!(p->rho0 > 0.0) || !std::isfinite(p->ax) || !std::isfinite(p->ay))
        return fail(LBM_E_PARAM, "rho0 must be positive and a finite");

    // Host-side validation first: no HIP call is made before the inputs are known to be good.
    lbm_ctx* c = new lbm_ctx();
    c->p = *p;
    c->stream = static_cast<hipStream_t>(stream);
    c->nx = uint32_t(p->nx);
    c->ny = uint32_t(p->ny);
    c->n = uint32_t(n64);
    c->ps = uint32_t((n64 + lbm::kChunk - 1) / lbm::kChunk * lbm::kChunk);
    lbm_status st = derive_globals(c);
    if (st != LBM_OK) {
        release(c);
        return st;
    }

    // --- flags and link validation (host) ---
    const uint32_t nx = c->nx, ny = c->ny, n = c->n;
    std::vector<uint8_t> flags(n, 0);
    for (uint32_t s = 0; s < n; ++s) flags[s] = solid[s] ? uint8_t(lbm::kSolid) : 0;
    auto neighbour = [&](int64_t x, int64_t y, int d, int64_t& out_site) -> bool {
        int64_t xn = x + kCx[d], yn = y + kCy[d];
        if (xn < 0 || xn >= int64_t(nx)) {
            if (!p->periodic_x) return false;
            xn = (xn + nx) % nx;
        }
        if (yn < 0 || yn >= int64_t(ny)) {
            if (!p->periodic_y) return false;
            yn = (yn + ny) % ny;
        }
        out_site = yn * nx + xn;
        return true;
    };
    std::vector<uint64_t> keys(static_cast<size_t>(n_links));
    for (int64_t k = 0; k < n_links; ++k) {
        const lbm_link& L = links[k];
        if (L.x < 0 || L.x >= p->nx || L.y < 0 || L.y >= p->ny || L.dir < 1 || L.dir > 8) {
            release(c);
            return fail(LBM_E_GEOMETRY, "link %lld: node (%d, %d) dir %d out of range", (long long)k, L.x, L.y, L.dir);
        }
        if (!(L.q > 0.0 && L.q <= 1.0) || !std::isfinite(L.ubx) || !std::isfinite(L.uby)) {
            release(c);
            return fail(LBM_E_GEOMETRY, "link %lld: q = %g not in (0, 1] or wall velocity not finite", (long long)k, L.q);
        }
        const int64_t s = int64_t(L.y) * nx + L.x;
        int64_t nb = -1;
        if (flags[s] == lbm::kSolid || !neighbour(L.x, L.y, L.dir, nb) || !solid[nb]) {
            release(c);
            return fail(LBM_E_GEOMETRY, "link %lld: (%d, %d) is not a fluid node with a solid neighbour along %d",
                        (long long)k, L.x, L.y, L.dir);
        }
        const uint8_t bit = uint8_t(1u << (L.dir - 1));
        if (flags[s] & bit) {
            release(c);
            return fail(LBM_E_GEOMETRY, "duplicate link at (%d, %d) dir %d", L.x, L.y, L.dir);
        }
        flags[s] |= bit;
        keys[size_t(k)] = (uint64_t(s) << 4) | uint64_t(L.dir);
    }
    int64_t n_fluid = 0;
    for (uint32_t y = 0; y < ny; ++y)
        for (uint32_t x = 0; x < nx; ++x) {
            const uint32_t s = y * nx + x;
            if (solid[s]) continue;
            ++n_fluid;
            int n_solid_nb = 0;
            for (int d = 1; d < 9; ++d) {
                int64_t nb = -1;
                if (!neighbour(x, y, d, nb)) {
                    release(c);
                    return fail(LBM_E_GEOMETRY, "fluid node (%u, %u) on a non-periodic edge: pad with solid", x, y);
                }
                if (solid[nb]) {
                    ++n_solid_nb;
                    if (!(flags[s] & (1u << (d - 1)))) {
                        release(c);
                        return fail(LBM_E_GEOMETRY, "missing wall link at (%u, %u) dir %d", x, y, d);
                    }
                }
            }
            if (n_solid_nb == 8) {
                release(c);
                return fail(LBM_E_GEOMETRY, "fluid node (%u, %u) has no fluid neighbour", x, y);
            }
        }
    c->n_fluid = n_fluid;
    c->n_links = n_links;

    // links sorted by (site, direction); chunk bases
    c->order.resize(size_t(n_links));
    for (int64_t k = 0; k < n_links; ++k) c->order[size_t(k)] = k;
    std::sort(c->order.begin(), c->order.end(), [&](int64_t a, int64_t b) { return keys[size_t(a)] < keys[size_t(b)]; });
    const uint32_t nchunks = (n + lbm::kChunk - 1) / lbm::kChunk;
    c->nchunks = nchunks;
    std::vector<int32_t>& chunk = c->chunk;
    chunk.assign(nchunks + 1, 0);
    {
        int64_t acc = 0;
        for (uint32_t ch = 0; ch < nchunks; ++ch) {
            chunk[ch] = int32_t(acc);
            const uint32_t e = std::min<uint32_t>(n, (ch + 1) * lbm::kChunk);
            for (uint32_t s = ch * lbm::kChunk; s < e; ++s)
                if (flags[s] != lbm::kSolid) acc += __builtin_popcount(flags[s]);
        }
        chunk[nchunks] = int32_t(acc);
    }
    std::vector<double> q(static_cast<size_t>(n_links)), ubx(static_cast<size_t>(n_links)), uby(static_cast<size_t>(n_links));
    std::vector<int32_t> dir(static_cast<size_t>(n_links));
    for (int64_t k = 0; k < n_links; ++k) {
        const lbm_link& L = links[c->order[size_t(k)]];
        q[size_t(k)] = L.q;
        ubx[size_t(k)] = L.ubx;
        uby[size_t(k)] = L.uby;
        dir[size_t(k)] = L.dir;
    }

    // LDS staging of one block's wall links; fall back to smaller blocks for link-dense geometries
    while (true) {
        c->lds_links = std::max<uint32_t>(c->max_links_per_block(c->block), 1u);
        if (lbm::step_lds_bytes(c->fp32(), c->lds_links) <= kMaxLds || c->block == 64) break;
        c->block /= 2;
    }
    if (lbm::step_lds_bytes(c->fp32(), c->lds_links) > kMaxLds) {
        release(c);
        return fail(LBM_E_GEOMETRY, "%u wall links in one 64-site chunk exceed the LDS staging area", c->lds_links);
    }

    // --- device allocations and uploads ---
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(LBM_E_HIP, "no HIP device available");
    }
    c->on_device = true;
    const size_t nl = size_t(std::max<int64_t>(n_links, 1));
    auto alloc = [&](void** ptr, size_t bytes) -> bool { return hipMalloc(ptr, bytes) == hipSuccess; };
    bool ok = alloc(reinterpret_cast<void**>(&c->d_flags), n) &&
              alloc(reinterpret_cast<void**>(&c->d_chunk), sizeof(int32_t) * (nchunks + 1)) &&
              alloc(reinterpret_cast<void**>(&c->d_coef64), sizeof(double) * 8 * nl) &&
              (!c->fp32() || alloc(reinterpret_cast<void**>(&c->d_coef32), sizeof(float) * 5 * nl)) &&
              alloc(&c->d_buf[0], c->pop_bytes()) && alloc(&c->d_buf[1], c->pop_bytes()) &&
              alloc(&c->d_link[0], c->link_bytes()) && alloc(&c->d_link[1], c->link_bytes()) &&
              alloc(reinterpret_cast<void**>(&c->d_uprev), sizeof(double) * 2 * n) &&
              alloc(reinterpret_cast<void**>(&c->d_partial), sizeof(double) * 3 * lbm::residual_blocks(n)) &&
              alloc(reinterpret_cast<void**>(&c->d_result), sizeof(double) * 4) &&
              hipHostMalloc(reinterpret_cast<void**>(&c->h_result), sizeof(double) * 4, hipHostMallocDefault) ==
                  hipSuccess;
    if (!ok) {
        release(c);
        return fail(LBM_E_NOMEM, "device allocation failed for %u sites", n);
    }
    double *d_q = nullptr, *d_ubx = nullptr, *d_uby = nullptr;
    int32_t* d_dir = nullptr;
    auto cleanup_tmp = [&]() {
        for (void* ptr : {static_cast<void*>(d_q), static_cast<void*>(d_ubx), static_cast<void*>(d_uby),
                          static_cast<void*>(d_dir)})
            if (ptr) ignore(hipFree(ptr));
    };
    if (!alloc(reinterpret_cast<void**>(&d_q), sizeof(double) * nl) ||
        !alloc(reinterpret_cast<void**>(&d_ubx), sizeof(double) * nl) ||
        !alloc(reinterpret_cast<void**>(&d_uby), sizeof(double) * nl) ||
        !alloc(reinterpret_cast<void**>(&d_dir), sizeof(int32_t) * nl)) {
        cleanup_tmp();
        release(c);
        return fail(LBM_E_NOMEM, "device allocation failed for %lld links", (long long)n_links);
    }
    hipError_t he = hipSuccess;
    auto H2D = [&](void* dst, const void* src, size_t bytes) {
        if (he == hipSuccess && bytes) he = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
    };
    H2D(c->d_flags, flags.data(), n);
    H2D(c->d_chunk, chunk.data(), sizeof(int32_t) * (nchunks + 1));
    H2D(d_q, q.data(), sizeof(double) * size_t(n_links));
    H2D(d_ubx, ubx.data(), sizeof(double) * size_t(n_links));
    H2D(d_uby, uby.data(), sizeof(double) * size_t(n_links));
    H2D(d_dir, dir.data(), sizeof(int32_t) * size_t(n_links));
    if (he == hipSuccess) {
        lbm::LinkInput in{d_q, d_ubx, d_uby, d_dir};
        lbm::PrecomputeArgs a{};
        a.tau_s = c->tau_s;
        a.L1 = c->L1;
        a.E = c->E;
        a.sq6pi = std::sqrt(6.0 / kPi);
        a.r_override = p->r_override;
        a.l_override = p->l_override;
        a.l_mode = p->l_mode;
        a.r_mode = p->r_mode;
        a.diffuse = p->diffuse;
        a.n_links = n_links;
        he = lbm::launch_precompute(in, a, c->d_coef64, c->fp32() ? c->d_coef32 : nullptr, c->stream);
    }
    std::vector<double> lrow(3 * nl);
    if (he == hipSuccess && n_links > 0) {
        for (int row = 0; row < 3 && he == hipSuccess; ++row)
            he = hipMemcpyAsync(lrow.data() + size_t(row) * nl, c->d_coef64 + size_t(row) * nl,
                                sizeof(double) * size_t(n_links), hipMemcpyDeviceToHost, c->stream);
    }
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    cleanup_tmp();
    if (he != hipSuccess) {
        release(c);
        return fail(LBM_E_HIP, "upload or precompute failed: %s", hipGetErrorString(he));
    }
    for (int64_t k = 0; k < n_links; ++k) {
        const double lraw = lrow[size_t(k)], l = lrow[nl + size_t(k)], r = lrow[2 * nl + size_t(k)];
        if (!(1.0 + l > 0.0) || !(r >= 0.0 && r <= 1.0)) {
            release(c);
            return fail(LBM_E_PARAM, "link %lld: l = %g, r = %g outside 1 + l > 0, 0 <= r <= 1",
                        (long long)c->order[size_t(k)], l, r);
        }
        if (l != lraw) ++c->n_clamped;
        const double g = q[size_t(k)];
        if (l < std::max(0.0, 2.0 * g - 1.0) || l > 2.0 * g) ++c->n_nonconvex;
    }
    st = lbm_init_rest(c);
    if (st != LBM_OK) {
        release(c);
        return st;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* ctx)
{
    release(ctx);
    return LBM_OK;
}

lbm_status lbm_get_info(const lbm_ctx* c, lbm_info* info)
{
    if (!c || !info) return fail(LBM_E_INVAL, "null argument");
    std::memset(info, 0, sizeof *info);
    info->tau_s = c->tau_s;
    info->tau_q = c->tau_q;
    info->E = c->E;
    info->E_max = c->E_max;
    info->L1 = c->L1;
    info->L2 = c->L2;
    info->nu = (c->tau_s - 0.5) / 3.0;
    info->n_sites = c->n;
    info->n_fluid = c->n_fluid;
    info->n_links = c->n_links;
    info->n_clamped = c->n_clamped;
    info->n_nonconvex = c->n_nonconvex;
    info->precision = c->p.precision;
    const int64_t sz = c->fp32() ? 4 : 8;
    const int64_t nchunks = (int64_t(c->n) + lbm::kChunk - 1) / lbm::kChunk;
    info->bytes_per_step = 18 * sz * c->n_fluid + 5 * sz * c->n_links + int64_t(c->n) + 4 * nchunks;
    info->steps = c->steps;
    return LBM_OK;
}

lbm_status lbm_link_coeffs(lbm_ctx* c, double* out)
{
    if (!c || (!out && c->n_links)) return fail(LBM_E_INVAL, "null argument");
    if (c->n_links == 0) return LBM_OK;
    DeviceGuard g(c->device);
    const size_t nl = size_t(c->n_links);
    std::vector<double> rows(8 * nl);
    HIP_TRY(hipMemcpyAsync(rows.data(), c->d_coef64, sizeof(double) * 8 * nl, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < nl; ++k)
        for (int r = 0; r < 8; ++r) out[size_t(c->order[k]) * 8 + size_t(r)] = rows[size_t(r) * nl + k];
    return LBM_OK;
}

lbm_status lbm_init_rest(lbm_ctx* c)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    DeviceGuard g(c->device);
    // deviations from the rest state are zero; both time levels and the recorded velocity
    HIP_TRY(lbm::launch_fill_zero(c->d_buf[0], c->pop_bytes(), c->stream));
    HIP_TRY(lbm::launch_fill_zero(c->d_buf[1], c->pop_bytes(), c->stream));
    HIP_TRY(lbm::launch_fill_zero(c->d_link[0], c->link_bytes(), c->stream));
    HIP_TRY(lbm::launch_fill_zero(c->d_link[1], c->link_bytes(), c->stream));
    HIP_TRY(lbm::launch_fill_zero(c->d_uprev, sizeof(double) * 2 * c->n, c->stream));
    c->cur = 0;
    c->steps = 0;
    c->uprev_valid = false;
    return LBM_OK;
}

lbm_status lbm_init_fields(lbm_ctx* c, const double* rho, const double* ux, const double* uy, int32_t device_ptrs)
{
    if (!c || !rho || !ux || !uy) return fail(LBM_E_INVAL, "null argument");
    DeviceGuard g(c->device);
    lbm_status st = lbm_init_rest(c);
    if (st != LBM_OK) return st;
    const double *dr = rho, *du = ux, *dv = uy;
    if (!device_ptrs) {
        if (!c->d_stage && hipMalloc(reinterpret_cast<void**>(&c->d_stage), sizeof(double) * 3 * c->n) != hipSuccess)
            return fail(LBM_E_NOMEM, "staging buffer");
        HIP_TRY(hipMemcpyAsync(c->d_stage, rho, sizeof(double) * c->n, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->d_stage + c->n, ux, sizeof(double) * c->n, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->d_stage + 2 * size_t(c->n), uy, sizeof(double) * c->n, hipMemcpyHostToDevice,
                               c->stream));
        dr = c->d_stage;
        du = c->d_stage + c->n;
        dv = c->d_stage + 2 * size_t(c->n);
    }
    HIP_TRY(lbm::launch_init_fields(c->fp32(), c->geo(), c->d_buf[0], c->d_link[0], dr, du, dv, c->p.rho0, c->p.ax,
                                    c->p.ay, c->stream));
    if (!device_ptrs) HIP_TRY(hipStreamSynchronize(c->stream));  // the host arrays may go away
    return LBM_OK;
}

extern "C++" template <typename T>
static lbm::StepArgs<T> step_args(const lbm_ctx* c, int src, int dst, const T* const* coef_rows)
{
    lbm::StepArgs<T> a{};
    a.g = c->geo();
    a.src = {static_cast<T*>(c->d_buf[src]), static_cast<T*>(c->d_link[src])};
    a.dst = {static_cast<T*>(c->d_buf[dst]), static_cast<T*>(c->d_link[dst])};
    a.coef = {coef_rows[0], coef_rows[1], coef_rows[2], coef_rows[3], coef_rows[4]};
    a.ux_out = c->d_uprev;
    a.uy_out = c->d_uprev + c->n;
    a.lds_links = c->lds_links;
    const double s_e = 1.0 / c->p.tau_e, s_eps = 1.0 / c->p.tau_eps, s_q = 1.0 / c->tau_q, s_s = 1.0 / c->tau_s;
    a.rho0 = T(c->p.rho0);
    a.ax = T(c->p.ax);
    a.ay = T(c->p.ay);
    a.s_e = T(s_e);
    a.s_eps = T(s_eps);
    a.s_q = T(s_q);
    a.s_s = T(s_s);
    a.c_e = T(1.0 - 0.5 * s_e);
    a.c_eps = T(1.0 - 0.5 * s_eps);
    a.c_q = T(1.0 - 0.5 * s_q);
    a.c_s = T(1.0 - 0.5 * s_s);
    return a;
}

static lbm_status step_once(lbm_ctx* c, bool write_u)
{
    const int src = c->cur, dst = 1 - c->cur;
    const bool node = c->p.diffuse == LBM_DIFFUSE_NODE;
    const size_t nl = size_t(std::max<int64_t>(c->n_links, 1));
    hipError_t e;
    if (c->fp32()) {
        const float* k32 = c->d_coef32;
        const float* rows[5] = {k32, k32 + nl, k32 + 2 * nl, k32 + 3 * nl, k32 + 4 * nl};
        e = lbm::launch_step_f32(step_args<float>(c, src, dst, rows), c->block, write_u, node, c->stream);
    } else {
        const double* k64 = c->d_coef64;
        const double* rows[5] = {k64 + 3 * nl, k64 + 4 * nl, k64 + 5 * nl, k64 + 6 * nl, k64 + 7 * nl};
        e = lbm::launch_step_f64(step_args<double>(c, src, dst, rows), c->block, write_u, node, c->stream);
    }
    if (e != hipSuccess) return fail(LBM_E_HIP, "step launch: %s", hipGetErrorString(e));
    c->cur = dst;
    ++c->steps;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    if (nsteps < 0) return fail(LBM_E_INVAL, "negative step count");
    if (nsteps == 0) return LBM_OK;
    DeviceGuard g(c->device);
    if (c->timing) HIP_TRY(hipEventRecord(c->ev0, c->stream));
    for (int64_t it = 0; it < nsteps; ++it) {
        // the last step records u(t) so that lbm_residual can compare it with u(t + 1)
        lbm_status st = step_once(c, it == nsteps - 1);
        if (st != LBM_OK) return st;
    }
    if (c->timing) {
        HIP_TRY(hipEventRecord(c->ev1, c->stream));
        c->have_timing = true;
        c->timed_steps = nsteps;
    }
    c->uprev_valid = true;
    return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx* c, double* rho, double* ux, double* uy, int32_t device_ptrs)
{
    if (!c || !rho || !ux || !uy) return fail(LBM_E_INVAL, "null argument");
    DeviceGuard g(c->device);
    if (device_ptrs) {
        HIP_TRY(lbm::launch_moments(c->fp32(), c->geo(), c->d_buf[c->cur], c->d_link[c->cur], rho, ux, uy, c->p.rho0,
                                    c->p.ax, c->p.ay, c->stream));
        return LBM_OK;
    }
    if (!c->d_stage && hipMalloc(reinterpret_cast<void**>(&c->d_stage), sizeof(double) * 3 * c->n) != hipSuccess)
        return fail(LBM_E_NOMEM, "staging buffer");
    double* s = c->d_stage;
    HIP_TRY(lbm::launch_moments(c->fp32(), c->geo(), c->d_buf[c->cur], c->d_link[c->cur], s, s + c->n,
                                s + 2 * size_t(c->n), c->p.rho0, c->p.ax, c->p.ay, c->stream));
    HIP_TRY(hipMemcpyAsync(rho, s, sizeof(double) * c->n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(ux, s + c->n, sizeof(double) * c->n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(uy, s + 2 * size_t(c->n), sizeof(double) * c->n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_residual(lbm_ctx* c, double* residual, double* mass)
{
    if (!c || !residual || !mass) return fail(LBM_E_INVAL, "null argument");
    DeviceGuard g(c->device);
    lbm::ReduceArgs a{};
    a.g = c->geo();
    a.pop = c->d_buf[c->cur];
    a.link = c->d_link[c->cur];
    a.ux_prev = c->d_uprev;
    a.uy_prev = c->d_uprev + c->n;
    a.partial = c->d_partial;
    a.rho0 = c->p.rho0;
    a.ax = c->p.ax;
    a.ay = c->p.ay;
    HIP_TRY(lbm::launch_residual(c->fp32(), a, c->d_result, c->stream));
    HIP_TRY(hipMemcpyAsync(c->h_result, c->d_result, sizeof(double) * 3, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const double s_du = c->h_result[0], s_u = c->h_result[1], s_dr = c->h_result[2];
    *mass = double(c->n_fluid) * c->p.rho0 + s_dr;
    *residual = c->uprev_valid ? std::sqrt(s_du / s_u) : HUGE_VAL;
    if (!std::isfinite(s_du) || !std::isfinite(s_u) || !std::isfinite(s_dr))
        return fail(LBM_E_UNSTABLE, "state is not finite after %lld steps", (long long)c->steps);
    return LBM_OK;
}

lbm_status lbm_set_stream(lbm_ctx* c, void* stream)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    DeviceGuard g(c->device);
    HIP_TRY(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    c->stream = static_cast<hipStream_t>(stream);
    return LBM_OK;
}

lbm_status lbm_synchronize(lbm_ctx* c)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    DeviceGuard g(c->device);
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_set_launch(lbm_ctx* c, int32_t block)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024)
        return fail(LBM_E_INVAL, "block %d not one of 64, 128, 256, 512, 1024", block);
    const uint32_t links = std::max<uint32_t>(c->max_links_per_block(block), 1u);
    if (lbm::step_lds_bytes(c->fp32(), links) > kMaxLds)
        return fail(LBM_E_INVAL, "block %d would stage %u wall links, more than the LDS limit", block, links);
    c->block = block;
    c->lds_links = links;
    return LBM_OK;
}

lbm_status lbm_set_timing(lbm_ctx* c, int32_t on)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    DeviceGuard g(c->device);
    if (on && !c->ev0) {
        HIP_TRY(hipEventCreate(&c->ev0));
        HIP_TRY(hipEventCreate(&c->ev1));
    }
    c->timing = on != 0;
    c->have_timing = false;
    return LBM_OK;
}

lbm_status lbm_last_step_ms(lbm_ctx* c, double* ms_total, int64_t* nsteps)
{
    if (!c || !ms_total || !nsteps) return fail(LBM_E_INVAL, "null argument");
    *ms_total = 0.0;
    *nsteps = 0;
    if (!c->have_timing) return LBM_OK;
    DeviceGuard g(c->device);
    HIP_TRY(hipEventSynchronize(c->ev1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    *ms_total = ms;
    *nsteps = c->timed_steps;
    return LBM_OK;
}

}  // extern "C"
