// Host-side validation, preparation and per-link precompute shared by the C ABI entry points.
#include "lbm_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

namespace lbm {

namespace {

thread_local std::string g_last_error;

constexpr double kPi = 3.14159265358979323846;
const int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

bool is_set(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

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

const char* last_error() { return g_last_error.c_str(); }

// Global parameters of the prescription, Sec. III.B and Sec. IV.
lbm_status derive_globals(const lbm_params& p, Globals& g)
{
    const double sq = std::sqrt(6.0 / kPi);
    g.tau_s = is_set(p.tau_s_override) ? p.tau_s_override : 0.5 + sq * p.kn * p.h;  // Eq. (tKnrela)
    if (!(g.tau_s > 0.5)) return fail(LBM_E_PARAM, "tau_s = %g must exceed 1/2", g.tau_s);
    g.L1 = std::isnan(p.L1) ? (2.0 - p.sigma) * (1.0 - 0.1817 * p.sigma) / p.sigma : p.L1;
    g.L2 = std::isnan(p.L2) ? 1.0 / kPi + 0.5 * g.L1 * g.L1 : p.L2;
    if (!std::isfinite(g.L1) || !std::isfinite(g.L2)) return fail(LBM_E_PARAM, "slip coefficients not finite");
    const double ts = g.tau_s, t2 = 2.0 * ts - 1.0;
    // Eq. (EqECond): tau_q > 1/2  <=>  E < E_max
    g.E_max = (kPi * ts * g.L2 - 3.0 * std::sqrt(kPi / 6.0) * g.L1) * t2 / (12.0 * ts) - 0.5;
    g.E = std::isnan(p.E) ? std::min(-0.65, g.E_max - 0.05) : p.E;
    // Eq. (NSliCoertstq)
    g.tau_q = is_set(p.tau_q_override)
                  ? p.tau_q_override
                  : (t2 * (ts * std::sqrt(6.0 * kPi) * g.L2 - g.L1) - 2.0 * sq * ts * (1.0 + 6.0 * g.E)) /
                        (8.0 * sq * ts + 4.0 * g.L1 * t2);
    if (!(g.tau_q > 0.5))
        return fail(LBM_E_PARAM, "tau_q = %g must exceed 1/2 (E = %g, bound %g)", g.tau_q, g.E, g.E_max);
    const double others[4] = {p.tau_rho, p.tau_e, p.tau_eps, p.tau_j};
    for (double t : others)
        if (!(t > 0.5)) return fail(LBM_E_PARAM, "relaxation time %g must exceed 1/2", t);
    return LBM_OK;
}


lbm_status check_params(const lbm_params& p, Globals& g)
{
    if (p.l_mode < 0 || p.l_mode > LBM_L_WALL_FIT || p.r_mode < 0 || p.r_mode > LBM_R_WALL_FIT || p.diffuse < 0 ||
        p.diffuse > 1 || p.precision < 0 || p.precision > 1)
        return fail(LBM_E_INVAL, "mode out of range");
    if (p.l_mode == LBM_L_WALL_FIT && p.r_mode != LBM_R_WALL_FIT)
        return fail(LBM_E_INVAL, "LBM_L_WALL_FIT needs LBM_R_WALL_FIT");
    if (!(p.rho0 > 0.0) || !std::isfinite(p.ax) || !std::isfinite(p.ay))
        return fail(LBM_E_PARAM, "rho0 must be positive and a finite");
    return derive_globals(p, g);
}

lbm_status prepare(const lbm_params* p, const uint8_t* solid, const lbm_link* links, int64_t n_links,
                   Prepared& out)
{
    if (!p || !solid || (n_links > 0 && !links) || n_links < 0) return fail(LBM_E_INVAL, "null or negative input");
    // the chunk table holds link offsets as int32
    if (n_links > INT32_MAX)
        return fail(LBM_E_INVAL, "%lld wall links exceed 2^31 - 1", (long long)n_links);
    if (p->nx <= 0 || p->ny <= 0) return fail(LBM_E_INVAL, "lattice size %d x %d", p->nx, p->ny);
    const uint64_t n64 = uint64_t(p->nx) * uint64_t(p->ny);
    if (n64 >= (uint64_t(1) << 31))
        return fail(LBM_E_INVAL, "lattice of %llu sites exceeds 2^31", (unsigned long long)n64);
    out.p = *p;
    lbm_status st = check_params(*p, out.g);
    if (st != LBM_OK) return st;

    const uint32_t nx = uint32_t(p->nx), ny = uint32_t(p->ny), n = uint32_t(n64);
    out.nx = nx;
    out.ny = ny;
    out.n = n;
    std::vector<uint8_t>& flags = out.flags;
    flags.assign(n, 0);
    for (uint32_t s = 0; s < n; ++s) flags[s] = solid[s] ? uint8_t(kSolid) : 0;
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
        if (L.x < 0 || L.x >= p->nx || L.y < 0 || L.y >= p->ny || L.dir < 1 || L.dir > 8)
            return fail(LBM_E_GEOMETRY, "link %lld: node (%d, %d) dir %d out of range", (long long)k, L.x, L.y, L.dir);
        if (!(L.q > 0.0 && L.q <= 1.0) || !std::isfinite(L.ubx) || !std::isfinite(L.uby))
            return fail(LBM_E_GEOMETRY, "link %lld: q = %g not in (0, 1] or wall velocity not finite", (long long)k,
                        L.q);
        const int64_t s = int64_t(L.y) * nx + L.x;
        int64_t nb = -1;
        if (flags[s] == kSolid || !neighbour(L.x, L.y, L.dir, nb) || !solid[nb])
            return fail(LBM_E_GEOMETRY, "link %lld: (%d, %d) is not a fluid node with a solid neighbour along %d",
                        (long long)k, L.x, L.y, L.dir);
        const uint8_t bit = uint8_t(1u << (L.dir - 1));
        if (flags[s] & bit) return fail(LBM_E_GEOMETRY, "duplicate link at (%d, %d) dir %d", L.x, L.y, L.dir);
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
                if (!neighbour(x, y, d, nb))
                    return fail(LBM_E_GEOMETRY, "fluid node (%u, %u) on a non-periodic edge: pad with solid", x, y);
                if (solid[nb]) {
                    ++n_solid_nb;
                    if (!(flags[s] & (1u << (d - 1))))
                        return fail(LBM_E_GEOMETRY, "missing wall link at (%u, %u) dir %d", x, y, d);
                }
            }
            if (n_solid_nb == 8) return fail(LBM_E_GEOMETRY, "fluid node (%u, %u) has no fluid neighbour", x, y);
        }
    out.n_fluid = n_fluid;
    out.n_links = n_links;

    // links sorted by (site, direction); chunk bases
    out.order.resize(size_t(n_links));
    for (int64_t k = 0; k < n_links; ++k) out.order[size_t(k)] = k;
    std::sort(out.order.begin(), out.order.end(),
              [&](int64_t a, int64_t b) { return keys[size_t(a)] < keys[size_t(b)]; });
    const uint32_t nchunks = (n + kChunk - 1) / kChunk;
    out.nchunks = nchunks;
    out.chunk.assign(nchunks + 1, 0);
    int64_t acc = 0;
    for (uint32_t ch = 0; ch < nchunks; ++ch) {
        out.chunk[ch] = int32_t(acc);
        const uint32_t e = std::min<uint32_t>(n, (ch + 1) * kChunk);
        for (uint32_t s = ch * kChunk; s < e; ++s)
            if (flags[s] != kSolid) acc += __builtin_popcount(flags[s]);
    }
    out.chunk[nchunks] = int32_t(acc);
    const size_t nl = static_cast<size_t>(n_links);
    out.q.resize(nl);
    out.ubx.resize(nl);
    out.uby.resize(nl);
    out.dir.resize(nl);
    for (size_t k = 0; k < nl; ++k) {
        const lbm_link& L = links[out.order[k]];
        out.q[k] = L.q;
        out.ubx[k] = L.ubx;
        out.uby[k] = L.uby;
        out.dir[k] = L.dir;
    }
    return LBM_OK;
}

lbm_status precompute_links(const Prepared& pr, double* coef64, float* coef32, int64_t stride, int64_t link_off,
                            hipStream_t stream, int32_t& n_clamped, int32_t& n_nonconvex)
{
    n_clamped = n_nonconvex = 0;
    const int64_t n_links = pr.n_links;
    if (n_links == 0) return LBM_OK;
    const size_t nl = size_t(n_links);
    double *d_q = nullptr, *d_ubx = nullptr, *d_uby = nullptr;
    int32_t* d_dir = nullptr;
    auto cleanup = [&]() {
        for (void* ptr : {static_cast<void*>(d_q), static_cast<void*>(d_ubx), static_cast<void*>(d_uby),
                          static_cast<void*>(d_dir)})
            if (ptr) ignore(hipFree(ptr));
    };
    if (hipMalloc(reinterpret_cast<void**>(&d_q), sizeof(double) * nl) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d_ubx), sizeof(double) * nl) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d_uby), sizeof(double) * nl) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d_dir), sizeof(int32_t) * nl) != hipSuccess) {
        cleanup();
        return fail(LBM_E_NOMEM, "device allocation failed for %lld links", (long long)n_links);
    }
    hipError_t he = hipSuccess;
    auto H2D = [&](void* dst, const void* src, size_t bytes) {
        if (he == hipSuccess) he = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
    };
    H2D(d_q, pr.q.data(), sizeof(double) * nl);
    H2D(d_ubx, pr.ubx.data(), sizeof(double) * nl);
    H2D(d_uby, pr.uby.data(), sizeof(double) * nl);
    H2D(d_dir, pr.dir.data(), sizeof(int32_t) * nl);
    if (he == hipSuccess) {
        LinkInput in{d_q, d_ubx, d_uby, d_dir};
        PrecomputeArgs a{};
        a.tau_s = pr.g.tau_s;
        a.tau_q = pr.g.tau_q;
        a.L1 = pr.g.L1;
        a.L2 = pr.g.L2;
        a.E = pr.g.E;
        a.sq6pi = std::sqrt(6.0 / kPi);
        a.r_override = pr.p.r_override;
        a.l_override = pr.p.l_override;
        a.l_mode = pr.p.l_mode;
        a.r_mode = pr.p.r_mode;
        a.diffuse = pr.p.diffuse;
        a.n_links = n_links;
        a.row_stride = stride;
        he = launch_precompute(in, a, coef64 + link_off, coef32 ? coef32 + link_off : nullptr, stream);
    }
    std::vector<double> lrow(3 * nl);
    for (int row = 0; row < 3 && he == hipSuccess; ++row)
        he = hipMemcpyAsync(lrow.data() + size_t(row) * nl, coef64 + size_t(row) * size_t(stride) + size_t(link_off),
                            sizeof(double) * nl, hipMemcpyDeviceToHost, stream);
    if (he == hipSuccess) he = hipStreamSynchronize(stream);
    cleanup();
    if (he != hipSuccess) return fail(LBM_E_HIP, "link upload or precompute failed: %s", hipGetErrorString(he));
    const bool wall_fit = pr.p.l_mode == LBM_L_WALL_FIT || pr.p.r_mode == LBM_R_WALL_FIT;
    const double lam = (pr.g.tau_s - 0.5) / std::sqrt(6.0 / kPi);
    if (wall_fit && !(pr.g.L1 > 0.0)) return fail(LBM_E_PARAM, "the wall-reading fit needs L1 > 0");
    for (size_t k = 0; k < nl; ++k) {
        const double lraw = lrow[k], l = lrow[nl + k], r = lrow[2 * nl + k];
        if (wall_fit && !(pr.q[k] < pr.g.tau_s - pr.g.L1 * lam))
            return fail(LBM_E_PARAM,
                        "link %lld: gamma = %g: the wall reading reaches the Kn term of the slip only for "
                        "gamma < tau_s - L1 Kn H = %g",
                        (long long)pr.order[k], pr.q[k], pr.g.tau_s - pr.g.L1 * lam);
        if (!(1.0 + l > 0.0) || !(r >= 0.0 && r <= 1.0))
            return fail(LBM_E_PARAM, "link %lld: l = %g, r = %g outside 1 + l > 0, 0 <= r <= 1",
                        (long long)pr.order[k], l, r);
        if (l != lraw) ++n_clamped;
        const double g = pr.q[k];
        if (l < std::max(0.0, 2.0 * g - 1.0) || l > 2.0 * g) ++n_nonconvex;
    }
    return LBM_OK;
}

}  // namespace lbm

extern "C" lbm_status lbm_params_comparison(lbm_params* p, int32_t scheme, double gamma_frozen)
{
    if (!p) return lbm::fail(LBM_E_INVAL, "null params");
    const double sq = std::sqrt(6.0 / lbm::kPi);
    const double ts = lbm::is_set(p->tau_s_override) ? p->tau_s_override : 0.5 + sq * p->kn * p->h;  // Eq. (tKnrela)
    if (!(ts > 0.5)) return lbm::fail(LBM_E_PARAM, "tau_s = %g must exceed 1/2", ts);
    const double L1 = std::isnan(p->L1) ? (2.0 - p->sigma) * (1.0 - 0.1817 * p->sigma) / p->sigma : p->L1;
    const double L2 = std::isnan(p->L2) ? 1.0 / lbm::kPi + 0.5 * L1 * L1 : p->L2;
    const double t2 = 2.0 * ts - 1.0;
    const double den = 4.0 * t2 * (2.0 * sq * ts + L1 * t2);
    double tq = 0.0;
    switch (scheme) {
    case LBM_SCHEME_PRESENT:
        p->l_mode = LBM_L_PAPER;
        p->r_mode = LBM_R_FROM_LEFF;
        p->tau_q_override = 0.0;
        return LBM_OK;
    case LBM_SCHEME_PREVIOUS: {
        if (!(gamma_frozen > 0.0 && gamma_frozen <= 1.0))
            return lbm::fail(LBM_E_INVAL, "frozen gamma %g outside (0, 1]", gamma_frozen);
        const double g = gamma_frozen;
        // Eq. (SliCoeffrtstqrD)
        tq = (L1 * t2 * (2.0 * ts * (6.0 * g - 1.0) + 1.0) +
              sq * ts * (L2 * lbm::kPi * t2 * t2 + 12.0 * g * g + 2.0 * t2 * (6.0 * g - 1.0))) /
             den;
        break;
    }
    case LBM_SCHEME_WALL_READING:
        p->l_mode = LBM_L_WALL_FIT;
        p->r_mode = LBM_R_WALL_FIT;
        p->diffuse = LBM_DIFFUSE_WALL;
        p->tau_q_override = 0.0;
        return LBM_OK;
    case LBM_SCHEME_HALFWAY_DBB:
        // Eq. (SliCoeffHata)
        tq = (L1 * t2 * (4.0 * ts + 1.0) + sq * ts * (L2 * lbm::kPi * t2 * t2 + 4.0 * t2 + 3.0)) / den;
        break;
    default:
        return lbm::fail(LBM_E_INVAL, "unknown scheme %d", scheme);
    }
    if (!(tq > 0.5)) return lbm::fail(LBM_E_PARAM, "tau_q = %g must exceed 1/2", tq);
    // l = 0; r = Eq. (SliCoeffrtsr) at l = 0, which is Eq. (SliCoeffrtsrD) = Eq. (SliCoeffHar)
    p->l_mode = LBM_L_ZERO;
    p->r_mode = LBM_R_FROM_LEFF;
    p->tau_q_override = tq;
    return LBM_OK;
}
