// Host side of liblbm: the single-lattice C ABI declared in include/lbm.h.
//
// lbm_create validates the problem statement (mask and wall-link table of Sec. III.A) and derives
// the global parameters of the prescription (Sec. III.B) on the host in fp64 (lbm_host.hip),
// uploads the mask as one flag byte per site and the links sorted by (site, direction), and runs
// the per-link fp64 precompute on the device.  lbm_step then launches only the fused step kernel.
#include <hip/hip_runtime.h>

#include <initializer_list>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_host.hpp"
#include "lbm_internal.hpp"

using lbm::DeviceGuard;
using lbm::fail;
using lbm::ignore;

namespace lbm {
const char* last_error();
}

struct lbm_ctx {
    lbm::Prepared pr;  // host copy: parameters, globals, chunk offsets, link order
    int device = 0;
    bool on_device = false;
    hipStream_t stream = nullptr;
    uint32_t ps = 0;  // population plane stride: sites rounded up to whole 64-site chunks
    int32_t n_clamped = 0, n_nonconvex = 0;
    uint8_t* d_flags = nullptr;
    int32_t* d_chunk = nullptr;
    double* d_coef64 = nullptr;            // 8 rows of n_links
    float* d_coef32 = nullptr;             // 5 rows of n_links (fp32 storage only)
    void* d_buf[2] = {nullptr, nullptr};   // population planes, two time levels
    void* d_link[2] = {nullptr, nullptr};  // per-link incoming populations, two time levels
    int cur = 0;
    uint32_t lds_links = 0;                // LDS link slots for the current block size
    double* d_uprev = nullptr;             // 2 n
    double* d_partial = nullptr;
    double* d_result = nullptr;            // 4
    double* h_result = nullptr;            // pinned, 4
    double* d_stage = nullptr;             // 3 n, for host-side moments and fields
    int64_t steps = 0;
    bool uprev_valid = false;
    int block = 256;
    int fuse = 1;             // time steps per launch of the step kernel: 1, or 2 (two-step kernel)
    int fuse_rows = 0;        // tile rows of the two-step kernel; 0 = not supported by this lattice
    uint32_t fuse_links = 0;  // LDS link slots of the two-step kernel (most wall links in one tile)
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool have_timing = false;
    int64_t timed_steps = 0;
    // lbm_step by graph replay: captured launch sequences, keyed by (steps, parity at the start,
    // whether the last launch records u), on a private capture stream; replayed on `stream`
    struct StepGraph {
        int64_t n;
        int cur, end_cur;
        bool last;
        hipGraphExec_t exec;
    };
    std::vector<StepGraph> graphs;
    bool use_graphs = true;
    hipStream_t capture = nullptr;
    void drop_graphs()
    {
        for (auto& g : graphs) ignore(hipGraphExecDestroy(g.exec));
        graphs.clear();
    }

    uint32_t n() const { return pr.n; }
    int64_t n_links() const { return pr.n_links; }
    bool fp32() const { return pr.p.precision == LBM_FP32_SHIFTED; }
    size_t pop_bytes() const { return (fp32() ? 4 : 8) * size_t(9) * ps; }
    size_t link_bytes() const { return (fp32() ? 4 : 8) * size_t(n_links() > 0 ? n_links() : 1); }
    lbm::Geo geo() const { return lbm::Geo{d_flags, d_chunk, pr.n, pr.nx, pr.ny, pr.nchunks, ps}; }
    // Most wall links in one 64 x rows tile of the two-step kernel (each tile row is one chunk).
    uint32_t max_links_per_tile(int rows) const
    {
        uint32_t best = 0;
        const uint32_t tiles_x = pr.nx / lbm::kFuseTX;
        for (uint32_t ty = 0; ty < pr.ny / uint32_t(rows); ++ty)
            for (uint32_t tx = 0; tx < tiles_x; ++tx) {
                uint32_t sum = 0;
                for (int r = 0; r < rows; ++r) {
                    const uint32_t ch = ((ty * rows + r) * pr.nx + tx * lbm::kFuseTX) / lbm::kChunk;
                    sum += uint32_t(pr.chunk[ch + 1] - pr.chunk[ch]);
                }
                best = std::max(best, sum);
            }
        return best;
    }
    // Tile heights of the two-step kernel in order of preference: fp32 blocks (two rows per wave)
    // are fastest with 4-row tiles, whose small blocks fit eight to a CU; fp64 with 8 rows, where
    // the LDS tile caps the blocks per CU anyway and taller tiles recompute fewer halo rows.
    std::array<int, 2> fusion_rows_order() const
    {
        return fp32() ? std::array<int, 2>{4, 8} : std::array<int, 2>{8, 4};
    }
    // Whether the two-step kernel can run with `rows` tile rows, and its LDS link slots.
    bool fusion_fits(int rows, uint32_t* links) const
    {
        if (pr.nx % lbm::kFuseTX != 0 || rows < 1 || pr.ny % uint32_t(rows) != 0) return false;
        const uint32_t l = std::max<uint32_t>(max_links_per_tile(rows), 1u);
        if (lbm::step2_lds_bytes(fp32(), rows, l) > lbm::kMaxLds) return false;
        *links = l;
        return true;
    }
    // Most wall links owned by one block of `blk` sites.
    uint32_t max_links_per_block(int blk) const
    {
        const uint32_t per = uint32_t(blk) / lbm::kChunk;
        uint32_t best = 0;
        for (uint32_t c0 = 0; c0 < pr.nchunks; c0 += per) {
            const uint32_t c1 = std::min(c0 + per, pr.nchunks);
            best = std::max(best, uint32_t(pr.chunk[c1] - pr.chunk[c0]));
        }
        return best;
    }
};

namespace {

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
                      static_cast<void*>(c->d_uprev), static_cast<void*>(c->d_partial),
                      static_cast<void*>(c->d_result), static_cast<void*>(c->d_stage)})
        if (ptr) ignore(hipFree(ptr));
    if (c->h_result) ignore(hipHostFree(c->h_result));
    if (c->ev0) ignore(hipEventDestroy(c->ev0));
    if (c->ev1) ignore(hipEventDestroy(c->ev1));
    c->drop_graphs();
    if (c->capture) ignore(hipStreamDestroy(c->capture));
    ignore(hipSetDevice(prev));
    delete c;
}

template <typename T>
lbm::StepArgs<T> step_args(const lbm_ctx* c, int src, int dst, const T* const* rows)
{
    lbm::StepArgs<T> a{};
    a.g = c->geo();
    a.src = {static_cast<T*>(c->d_buf[src]), static_cast<T*>(c->d_link[src])};
    a.dst = {static_cast<T*>(c->d_buf[dst]), static_cast<T*>(c->d_link[dst])};
    a.coef = {rows[0], rows[1], rows[2], rows[3], rows[4]};
    a.ux_out = c->d_uprev;
    a.uy_out = c->d_uprev + c->n();
    a.lds_links = c->lds_links;
    const lbm::Phys<T> ph = lbm::make_phys<T>(c->pr.p, c->pr.g);
    a.rho0 = ph.rho0;
    a.ax = ph.ax;
    a.ay = ph.ay;
    a.s_e = ph.s_e;
    a.s_eps = ph.s_eps;
    a.s_q = ph.s_q;
    a.s_s = ph.s_s;
    a.c_e = ph.c_e;
    a.c_eps = ph.c_eps;
    a.c_q = ph.c_q;
    a.c_s = ph.c_s;
    return a;
}

lbm_status step_once(lbm_ctx* c, bool write_u)
{
    const int src = c->cur, dst = 1 - c->cur;
    const bool node = c->pr.p.diffuse == LBM_DIFFUSE_NODE;
    const size_t nl = size_t(std::max<int64_t>(c->n_links(), 1));
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

// Two time steps in one launch of the two-step kernel (same results as two step_once calls).
lbm_status step_pair(lbm_ctx* c, bool write_u)
{
    const int src = c->cur, dst = 1 - c->cur;
    const bool node = c->pr.p.diffuse == LBM_DIFFUSE_NODE;
    const size_t nl = size_t(std::max<int64_t>(c->n_links(), 1));
    hipError_t e;
    if (c->fp32()) {
        const float* k32 = c->d_coef32;
        const float* rows[5] = {k32, k32 + nl, k32 + 2 * nl, k32 + 3 * nl, k32 + 4 * nl};
        lbm::StepArgs<float> a = step_args<float>(c, src, dst, rows);
        a.lds_links = c->fuse_links;
        e = lbm::launch_step2_f32(a, c->fuse_rows, write_u, node, c->stream);
    } else {
        const double* k64 = c->d_coef64;
        const double* rows[5] = {k64 + 3 * nl, k64 + 4 * nl, k64 + 5 * nl, k64 + 6 * nl, k64 + 7 * nl};
        lbm::StepArgs<double> a = step_args<double>(c, src, dst, rows);
        a.lds_links = c->fuse_links;
        e = lbm::launch_step2_f64(a, c->fuse_rows, write_u, node, c->stream);
    }
    if (e != hipSuccess) return fail(LBM_E_HIP, "two-step launch: %s", hipGetErrorString(e));
    c->cur = dst;
    c->steps += 2;
    return LBM_OK;
}

}  // namespace

extern "C" {

int32_t lbm_version(void) { return 10100; }

const char* lbm_last_error(void) { return lbm::last_error(); }

lbm_status lbm_params_default(lbm_params* p)
{
    if (!p) return fail(LBM_E_INVAL, "null params");
    std::memset(p, 0, sizeof *p);
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
    // Host-side validation first: no HIP call is made before the inputs are known to be good.
    lbm_ctx* c = new lbm_ctx();
    lbm_status st = lbm::prepare(p, solid, links, n_links, c->pr);
    if (st != LBM_OK) {
        release(c);
        return st;
    }
    c->stream = static_cast<hipStream_t>(stream);
    const uint32_t n = c->n();
    c->ps = (n + lbm::kChunk - 1) / lbm::kChunk * lbm::kChunk;
    // LDS staging of one block's wall links; fall back to smaller blocks for link-dense geometries
    while (true) {
        c->lds_links = std::max<uint32_t>(c->max_links_per_block(c->block), 1u);
        if (lbm::step_lds_bytes(c->fp32(), c->lds_links) <= lbm::kMaxLds || c->block == 64) break;
        c->block /= 2;
    }
    if (lbm::step_lds_bytes(c->fp32(), c->lds_links) > lbm::kMaxLds) {
        release(c);
        return fail(LBM_E_GEOMETRY, "%u wall links in one 64-site chunk exceed the LDS staging area", c->lds_links);
    }
    // two time steps per launch by default where the lattice tiles into 64 x rows blocks (half the
    // HBM traffic per step; faster in both precisions)
    for (int rows : c->fusion_rows_order()) {
        uint32_t links = 0;
        if (c->fusion_fits(rows, &links)) {
            c->fuse = 2;
            c->fuse_rows = rows;
            c->fuse_links = links;
            break;
        }
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
              alloc(reinterpret_cast<void**>(&c->d_chunk), sizeof(int32_t) * (c->pr.nchunks + 1)) &&
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
    hipError_t he = hipMemcpyAsync(c->d_flags, c->pr.flags.data(), n, hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess)
        he = hipMemcpyAsync(c->d_chunk, c->pr.chunk.data(), sizeof(int32_t) * (c->pr.nchunks + 1),
                            hipMemcpyHostToDevice, c->stream);
    if (he != hipSuccess) {
        release(c);
        return fail(LBM_E_HIP, "upload failed: %s", hipGetErrorString(he));
    }
    st = lbm::precompute_links(c->pr, c->d_coef64, c->fp32() ? c->d_coef32 : nullptr, int64_t(nl), 0, c->stream,
                               c->n_clamped, c->n_nonconvex);
    if (st == LBM_OK) st = lbm_init_rest(c);
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
    info->tau_s = c->pr.g.tau_s;
    info->tau_q = c->pr.g.tau_q;
    info->E = c->pr.g.E;
    info->E_max = c->pr.g.E_max;
    info->L1 = c->pr.g.L1;
    info->L2 = c->pr.g.L2;
    info->nu = (c->pr.g.tau_s - 0.5) / 3.0;
    info->n_sites = c->n();
    info->n_fluid = c->pr.n_fluid;
    info->n_links = c->n_links();
    info->n_clamped = c->n_clamped;
    info->n_nonconvex = c->n_nonconvex;
    info->precision = c->pr.p.precision;
    const int64_t sz = c->fp32() ? 4 : 8;
    info->bytes_per_step = 18 * sz * c->pr.n_fluid + (5 + 5 * sz) * c->n_links() + int64_t(c->n());
    info->steps = c->steps;
    info->steps_per_launch = c->fuse;
    return LBM_OK;
}

lbm_status lbm_link_coeffs(lbm_ctx* c, double* out)
{
    if (!c || (!out && c->n_links())) return fail(LBM_E_INVAL, "null argument");
    if (c->n_links() == 0) return LBM_OK;
    DeviceGuard g(c->device);
    const size_t nl = size_t(c->n_links());
    std::vector<double> rows(8 * nl);
    LBM_HIP_TRY(hipMemcpyAsync(rows.data(), c->d_coef64, sizeof(double) * 8 * nl, hipMemcpyDeviceToHost, c->stream));
    LBM_HIP_TRY(hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < nl; ++k)
        for (int r = 0; r < 8; ++r) out[size_t(c->pr.order[k]) * 8 + size_t(r)] = rows[size_t(r) * nl + k];
    return LBM_OK;
}

lbm_status lbm_init_rest(lbm_ctx* c)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    DeviceGuard g(c->device);
    // deviations from the rest state are zero; both time levels and the recorded velocity
    LBM_HIP_TRY(lbm::launch_fill_zero(c->d_buf[0], c->pop_bytes(), c->stream));
    LBM_HIP_TRY(lbm::launch_fill_zero(c->d_buf[1], c->pop_bytes(), c->stream));
    LBM_HIP_TRY(lbm::launch_fill_zero(c->d_link[0], c->link_bytes(), c->stream));
    LBM_HIP_TRY(lbm::launch_fill_zero(c->d_link[1], c->link_bytes(), c->stream));
    LBM_HIP_TRY(lbm::launch_fill_zero(c->d_uprev, sizeof(double) * 2 * c->n(), c->stream));
    c->cur = 0;
    c->steps = 0;
    c->uprev_valid = false;
    return LBM_OK;
}

namespace {
lbm_status init_fields(lbm_ctx* c, const double* rho, const double* ux, const double* uy, int32_t device_ptrs,
                       double neq_tau)
{
    if (!c || !rho || !ux || !uy) return fail(LBM_E_INVAL, "null argument");
    DeviceGuard g(c->device);
    lbm_status st = lbm_init_rest(c);
    if (st != LBM_OK) return st;
    const uint32_t n = c->n();
    const double *dr = rho, *du = ux, *dv = uy;
    if (!device_ptrs) {
        if (!c->d_stage && hipMalloc(reinterpret_cast<void**>(&c->d_stage), sizeof(double) * 3 * n) != hipSuccess)
            return fail(LBM_E_NOMEM, "staging buffer");
        LBM_HIP_TRY(hipMemcpyAsync(c->d_stage, rho, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
        LBM_HIP_TRY(hipMemcpyAsync(c->d_stage + n, ux, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
        LBM_HIP_TRY(hipMemcpyAsync(c->d_stage + 2 * size_t(n), uy, sizeof(double) * n, hipMemcpyHostToDevice,
                                   c->stream));
        dr = c->d_stage;
        du = c->d_stage + n;
        dv = c->d_stage + 2 * size_t(n);
    }
    LBM_HIP_TRY(lbm::launch_init_fields(c->fp32(), c->geo(), c->d_buf[0], c->d_link[0], dr, du, dv, c->pr.p.rho0,
                                        c->pr.p.ax, c->pr.p.ay, neq_tau, c->stream));
    if (!device_ptrs) LBM_HIP_TRY(hipStreamSynchronize(c->stream));  // the host arrays may go away
    return LBM_OK;
}
}  // namespace

lbm_status lbm_init_fields(lbm_ctx* c, const double* rho, const double* ux, const double* uy, int32_t device_ptrs)
{
    return init_fields(c, rho, ux, uy, device_ptrs, 0.0);
}

lbm_status lbm_init_fields_neq(lbm_ctx* c, const double* rho, const double* ux, const double* uy, int32_t device_ptrs)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    return init_fields(c, rho, ux, uy, device_ptrs, c->pr.g.tau_s);
}

// The launches of n steps from the current time level; the last launch records u(t) for
// lbm_residual when `last` is set.
lbm_status run_steps(lbm_ctx* c, int64_t n, bool last)
{
    for (int64_t it = 0; it < n;) {
        const int64_t left = n - it;
        lbm_status st;
        if (c->fuse == 2 && left >= 2) {
            st = step_pair(c, last && left == 2);
            it += 2;
        } else {
            st = step_once(c, last && left == 1);
            it += 1;
        }
        if (st != LBM_OK) return st;
    }
    return LBM_OK;
}

// n steps by replaying a captured graph of run_steps(n, last) (captured at first use on the
// private capture stream; the host-side state is restored after capture and advanced as the
// replay advances it).  A capture failure switches the context to eager launches for good.
lbm_status graph_steps(lbm_ctx* c, int64_t n, bool last)
{
    lbm_ctx::StepGraph* g = nullptr;
    for (auto& e : c->graphs)
        if (e.n == n && e.cur == c->cur && e.last == last) g = &e;
    if (!g) {
        if (!c->capture && hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) {
            c->capture = nullptr;
            c->use_graphs = false;
            return run_steps(c, n, last);
        }
        if (c->graphs.size() >= 16) c->drop_graphs();
        const int cur0 = c->cur;
        const int64_t steps0 = c->steps;
        hipStream_t user = c->stream;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        bool ok = hipStreamBeginCapture(c->capture, hipStreamCaptureModeRelaxed) == hipSuccess;
        if (ok) {
            c->stream = c->capture;
            const lbm_status st = run_steps(c, n, last);
            c->stream = user;
            ok = hipStreamEndCapture(c->capture, &graph) == hipSuccess && st == LBM_OK && graph;
        }
        ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) ignore(hipGraphDestroy(graph));
        const int end_cur = c->cur;
        c->cur = cur0;
        c->steps = steps0;
        ignore(hipGetLastError());
        if (!ok) {
            if (exec) ignore(hipGraphExecDestroy(exec));
            c->use_graphs = false;
            return run_steps(c, n, last);
        }
        c->graphs.push_back(lbm_ctx::StepGraph{n, cur0, end_cur, last, exec});
        g = &c->graphs.back();
    }
    if (hipGraphLaunch(g->exec, c->stream) != hipSuccess) return fail(LBM_E_HIP, "step graph launch failed");
    c->cur = g->end_cur;
    c->steps += n;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    if (nsteps < 0) return fail(LBM_E_INVAL, "negative step count");
    if (nsteps == 0) return LBM_OK;
    DeviceGuard g(c->device);
    if (c->timing) LBM_HIP_TRY(hipEventRecord(c->ev0, c->stream));
    lbm_status st = LBM_OK;
    if (c->use_graphs && nsteps >= 4) {
        // graphs of at most 256 steps (an even count keeps the time-level parity of every launch
        // sequence but the last), the last one recording u
        constexpr int64_t kGraphSteps = 256;
        int64_t left = nsteps;
        while (st == LBM_OK && left > kGraphSteps) {
            st = graph_steps(c, kGraphSteps, false);
            left -= kGraphSteps;
        }
        if (st == LBM_OK) st = c->use_graphs ? graph_steps(c, left, true) : run_steps(c, left, true);
    } else {
        st = run_steps(c, nsteps, true);
    }
    if (st != LBM_OK) return st;
    if (c->timing) {
        LBM_HIP_TRY(hipEventRecord(c->ev1, c->stream));
        c->have_timing = true;
        c->timed_steps = nsteps;
    }
    c->uprev_valid = true;
    return LBM_OK;
}

lbm_status lbm_set_graphs(lbm_ctx* c, int32_t on)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    DeviceGuard g(c->device);
    c->drop_graphs();
    c->use_graphs = on != 0;
    return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx* c, double* rho, double* ux, double* uy, int32_t device_ptrs)
{
    if (!c || !rho || !ux || !uy) return fail(LBM_E_INVAL, "null argument");
    DeviceGuard g(c->device);
    const uint32_t n = c->n();
    if (device_ptrs) {
        LBM_HIP_TRY(lbm::launch_moments(c->fp32(), c->geo(), c->d_buf[c->cur], c->d_link[c->cur], rho, ux, uy,
                                        c->pr.p.rho0, c->pr.p.ax, c->pr.p.ay, c->stream));
        return LBM_OK;
    }
    if (!c->d_stage && hipMalloc(reinterpret_cast<void**>(&c->d_stage), sizeof(double) * 3 * n) != hipSuccess)
        return fail(LBM_E_NOMEM, "staging buffer");
    double* s = c->d_stage;
    LBM_HIP_TRY(lbm::launch_moments(c->fp32(), c->geo(), c->d_buf[c->cur], c->d_link[c->cur], s, s + n,
                                    s + 2 * size_t(n), c->pr.p.rho0, c->pr.p.ax, c->pr.p.ay, c->stream));
    LBM_HIP_TRY(hipMemcpyAsync(rho, s, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    LBM_HIP_TRY(hipMemcpyAsync(ux, s + n, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    LBM_HIP_TRY(hipMemcpyAsync(uy, s + 2 * size_t(n), sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    LBM_HIP_TRY(hipStreamSynchronize(c->stream));
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
    a.uy_prev = c->d_uprev + c->n();
    a.partial = c->d_partial;
    a.rho0 = c->pr.p.rho0;
    a.ax = c->pr.p.ax;
    a.ay = c->pr.p.ay;
    LBM_HIP_TRY(lbm::launch_residual(c->fp32(), a, c->d_result, c->stream));
    LBM_HIP_TRY(hipMemcpyAsync(c->h_result, c->d_result, sizeof(double) * 3, hipMemcpyDeviceToHost, c->stream));
    LBM_HIP_TRY(hipStreamSynchronize(c->stream));
    const double s_du = c->h_result[0], s_u = c->h_result[1], s_dr = c->h_result[2];
    *mass = double(c->pr.n_fluid) * c->pr.p.rho0 + s_dr;
    *residual = c->uprev_valid ? std::sqrt(s_du / s_u) : HUGE_VAL;
    if (!std::isfinite(s_du) || !std::isfinite(s_u) || !std::isfinite(s_dr))
        return fail(LBM_E_UNSTABLE, "state is not finite after %lld steps", (long long)c->steps);
    return LBM_OK;
}

lbm_status lbm_set_stream(lbm_ctx* c, void* stream)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    DeviceGuard g(c->device);
    LBM_HIP_TRY(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    c->stream = static_cast<hipStream_t>(stream);
    return LBM_OK;
}

lbm_status lbm_synchronize(lbm_ctx* c)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    DeviceGuard g(c->device);
    LBM_HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_stream_copy(void* dst, const void* src, int64_t bytes, void* stream)
{
    if (!dst || !src || bytes < 0) return fail(LBM_E_INVAL, "null pointer or negative size");
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src) | uint64_t(bytes)) & 15u)
        return fail(LBM_E_INVAL, "pointers and size must be multiples of 16 bytes");
    LBM_HIP_TRY(lbm::launch_stream_copy(dst, src, uint64_t(bytes), static_cast<hipStream_t>(stream)));
    return LBM_OK;
}

lbm_status lbm_set_launch(lbm_ctx* c, int32_t block)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024)
        return fail(LBM_E_INVAL, "block %d not one of 64, 128, 256, 512, 1024", block);
    const uint32_t links = std::max<uint32_t>(c->max_links_per_block(block), 1u);
    if (lbm::step_lds_bytes(c->fp32(), links) > lbm::kMaxLds)
        return fail(LBM_E_INVAL, "block %d would stage %u wall links, more than the LDS limit", block, links);
    c->block = block;
    c->drop_graphs();
    c->lds_links = links;
    return LBM_OK;
}

lbm_status lbm_set_fusion(lbm_ctx* c, int32_t steps_per_launch, int32_t rows)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    c->drop_graphs();
    if (steps_per_launch == 1) {
        c->fuse = 1;
        return LBM_OK;
    }
    if (steps_per_launch != 2) return fail(LBM_E_INVAL, "steps per launch must be 1 or 2, not %d", steps_per_launch);
    if (rows != 0 && rows != 4 && rows != 8) return fail(LBM_E_INVAL, "tile rows %d not one of 4, 8", rows);
    const std::array<int, 2> order = c->fusion_rows_order();
    const std::array<int, 2> cand = rows ? std::array<int, 2>{rows, rows} : order;
    for (int r : cand) {
        uint32_t links = 0;
        if (c->fusion_fits(r, &links)) {
            c->fuse = 2;
            c->fuse_rows = r;
            c->fuse_links = links;
            return LBM_OK;
        }
    }
    return fail(LBM_E_INVAL, "two-step kernel needs nx %% 64 == 0, ny %% rows == 0 and a tile's wall links in "
                "LDS (nx %u, ny %u)", c->pr.nx, c->pr.ny);
}

lbm_status lbm_set_timing(lbm_ctx* c, int32_t on)
{
    if (!c) return fail(LBM_E_INVAL, "null context");
    DeviceGuard g(c->device);
    if (on && !c->ev0) {
        LBM_HIP_TRY(hipEventCreate(&c->ev0));
        LBM_HIP_TRY(hipEventCreate(&c->ev1));
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
    LBM_HIP_TRY(hipEventSynchronize(c->ev1));
    float ms = 0.0f;
    LBM_HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    *ms_total = ms;
    *nsteps = c->timed_steps;
    return LBM_OK;
}

}  // extern "C"
