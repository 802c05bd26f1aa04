// Batched lattices (include/lbm.h, lbm_batch_*): many independent instances of uneven size in one
// site space, advanced by one persistent kernel launch per step and replayed from HIP graphs.
//
// Layout: instance i occupies sites [off_i, off_i + n_i) of a shared site space (off_i a multiple
// of kPad so that every tile of every launch shape starts inside one instance); the nine planes,
// the flag bytes, the chunk link offsets and the recorded velocities span the whole space; link
// arrays and coefficients are concatenated, instance by instance, in (site, direction) order.
//
// Scheduling: a host list of active tiles (instance, local start) lives in device memory together
// with its length.  The persistent kernel reads the length at launch and strides over the list, so
// graphs captured once stay valid when instances retire (only the list shrinks).  Retired
// instances keep their state in the buffer that held it when they retired.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_host.hpp"
#include "lbm_internal.hpp"

using lbm::DeviceGuard;
using lbm::fail;
using lbm::ignore;

namespace {
constexpr uint32_t kPad = 1024;  // instance offsets are multiples of the largest tile
constexpr int kFloorWindow = 50;
constexpr double kFloorRatio = 0.995;
constexpr double kFloorBelow = 1e-5;
}  // namespace

struct lbm_batch {
    int32_t n_inst = 0;
    bool fp32 = false, node = true;
    int device = 0;
    bool on_device = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<lbm::Prepared> pr;
    std::vector<uint32_t> off;
    std::vector<int64_t> link_off;
    std::vector<int32_t> n_clamped, n_nonconvex;
    uint32_t ps = 0;  // sites in the batch site space
    int64_t total_links = 0;
    std::vector<int32_t> chunk;  // global chunk table, ps / 64 + 1 entries
    uint8_t* d_flags = nullptr;
    int32_t* d_chunk = nullptr;
    double* d_coef64 = nullptr;
    float* d_coef32 = nullptr;
    void* d_buf[2] = {nullptr, nullptr};
    void* d_link[2] = {nullptr, nullptr};
    double* d_uprev = nullptr;
    void* d_inst = nullptr;
    lbm::TileRef* d_tiles = nullptr;
    uint32_t* d_n_active = nullptr;
    uint32_t* d_tile_begin = nullptr;
    double* d_partial = nullptr;
    double* d_result = nullptr;
    double* h_result = nullptr;
    uint32_t tile_capacity = 0;
    // state
    int cur = 0;
    std::vector<uint8_t> active;
    std::vector<int> inst_cur;
    std::vector<int64_t> steps;
    std::vector<uint8_t> uvalid;
    std::vector<double> last_res, last_mass;
    // launch
    lbm_batch_launch launch{256, 10, 4, 0};
    uint32_t lds_links = 1;
    uint32_t n_active_tiles = 0;
    std::vector<int32_t> active_list;  // active instances in tile order
    int n_cu = 1;
    hipGraphExec_t graph[2] = {nullptr, nullptr};

    size_t esize() const { return fp32 ? 4 : 8; }
    size_t pop_bytes() const { return esize() * 9 * size_t(ps); }
    size_t link_bytes() const { return esize() * size_t(std::max<int64_t>(total_links, 1)); }
    int64_t link_stride() const { return std::max<int64_t>(total_links, 1); }
};

namespace {

void drop_graphs(lbm_batch* b)
{
    for (hipGraphExec_t& g : b->graph)
        if (g) {
            ignore(hipGraphExecDestroy(g));
            g = nullptr;
        }
}

void release(lbm_batch* b)
{
    if (!b) return;
    if (b->on_device) {
        int prev = 0;
        ignore(hipGetDevice(&prev));
        ignore(hipSetDevice(b->device));
        ignore(hipStreamSynchronize(b->stream));
        drop_graphs(b);
        for (void* ptr : {static_cast<void*>(b->d_flags), static_cast<void*>(b->d_chunk),
                          static_cast<void*>(b->d_coef64), static_cast<void*>(b->d_coef32), b->d_buf[0], b->d_buf[1],
                          b->d_link[0], b->d_link[1], static_cast<void*>(b->d_uprev), b->d_inst,
                          static_cast<void*>(b->d_tiles), static_cast<void*>(b->d_n_active),
                          static_cast<void*>(b->d_tile_begin), static_cast<void*>(b->d_partial),
                          static_cast<void*>(b->d_result)})
            if (ptr) ignore(hipFree(ptr));
        if (b->h_result) ignore(hipHostFree(b->h_result));
        if (b->own_stream) ignore(hipStreamDestroy(b->stream));
        ignore(hipSetDevice(prev));
    }
    delete b;
}

// Most wall links in one tile of `blk` sites, over every instance.
uint32_t max_links_per_tile(const lbm_batch* b, int blk)
{
    uint32_t best = 1;
    const uint32_t per = uint32_t(blk) / lbm::kChunk;
    for (int32_t i = 0; i < b->n_inst; ++i) {
        const lbm::Prepared& p = b->pr[i];
        for (uint32_t c0 = 0; c0 < p.nchunks; c0 += per) {
            const uint32_t c1 = std::min(c0 + per, p.nchunks);
            best = std::max(best, uint32_t(p.chunk[c1] - p.chunk[c0]));
        }
    }
    return best;
}

uint32_t tiles_of(const lbm_batch* b, int32_t i, int blk) { return (b->pr[i].n + uint32_t(blk) - 1) / uint32_t(blk); }

// Rebuilds the active tile list for the current block size and active set (device copy and length).
lbm_status rebuild_tiles(lbm_batch* b)
{
    const int blk = b->launch.block;
    std::vector<lbm::TileRef> tiles;
    std::vector<uint32_t> begin;
    b->active_list.clear();
    for (int32_t i = 0; i < b->n_inst; ++i) {
        if (!b->active[i]) continue;
        b->active_list.push_back(i);
        begin.push_back(uint32_t(tiles.size()));
        const uint32_t nt = tiles_of(b, i, blk);
        for (uint32_t t = 0; t < nt; ++t) tiles.push_back(lbm::TileRef{uint32_t(i), t * uint32_t(blk)});
    }
    begin.push_back(uint32_t(tiles.size()));
    b->n_active_tiles = uint32_t(tiles.size());
    if (!tiles.empty())
        LBM_HIP_TRY(hipMemcpyAsync(b->d_tiles, tiles.data(), sizeof(lbm::TileRef) * tiles.size(), hipMemcpyHostToDevice,
                                   b->stream));
    LBM_HIP_TRY(hipMemcpyAsync(b->d_tile_begin, begin.data(), sizeof(uint32_t) * begin.size(), hipMemcpyHostToDevice,
                               b->stream));
    LBM_HIP_TRY(hipMemcpyAsync(b->d_n_active, &b->n_active_tiles, sizeof(uint32_t), hipMemcpyHostToDevice, b->stream));
    // the host vectors go out of scope: finish the copies first
    LBM_HIP_TRY(hipStreamSynchronize(b->stream));
    return LBM_OK;
}

uint32_t grid_of(const lbm_batch* b)
{
    uint32_t all = 0;
    for (int32_t i = 0; i < b->n_inst; ++i) all += tiles_of(b, i, b->launch.block);
    if (b->launch.blocks_per_cu <= 0) return std::max(all, 1u);
    return std::max(1u, std::min(all, uint32_t(b->n_cu * b->launch.blocks_per_cu)));
}

template <typename T>
lbm::BatchArgs<T> batch_args(const lbm_batch* b, int src, int dst)
{
    lbm::BatchArgs<T> a{};
    const int64_t st = b->link_stride();
    a.flags = b->d_flags;
    a.chunk_base = b->d_chunk;
    a.src = {static_cast<T*>(b->d_buf[src]), static_cast<T*>(b->d_link[src])};
    a.dst = {static_cast<T*>(b->d_buf[dst]), static_cast<T*>(b->d_link[dst])};
    if (b->fp32) {
        const T* k = reinterpret_cast<const T*>(b->d_coef32);
        a.coef = {k, k + st, k + 2 * st, k + 3 * st, k + 4 * st};
    } else {
        const T* k = reinterpret_cast<const T*>(b->d_coef64);
        a.coef = {k + 3 * st, k + 4 * st, k + 5 * st, k + 6 * st, k + 7 * st};
    }
    a.ux_out = b->d_uprev;
    a.uy_out = b->d_uprev + b->ps;
    a.inst = static_cast<const lbm::BatchInst<T>*>(b->d_inst);
    a.tiles = b->d_tiles;
    a.n_active = b->d_n_active;
    a.ps = b->ps;
    a.lds_links = b->lds_links;
    return a;
}

hipError_t launch_one(lbm_batch* b, int src, int dst, bool write_u)
{
    const uint32_t grid = grid_of(b);
    if (b->fp32)
        return lbm::launch_step_batch_f32(batch_args<float>(b, src, dst), b->launch.block, grid, write_u, b->node,
                                          b->stream);
    return lbm::launch_step_batch_f64(batch_args<double>(b, src, dst), b->launch.block, grid, write_u, b->node,
                                      b->stream);
}

// Graph of graph_steps steps starting from buffer `parity` (ends there again: the count is even);
// the last step records u for the residual.
lbm_status capture(lbm_batch* b, int parity)
{
    hipGraph_t g = nullptr;
    LBM_HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    int src = parity;
    for (int s = 0; s < b->launch.graph_steps && e == hipSuccess; ++s) {
        e = launch_one(b, src, 1 - src, s == b->launch.graph_steps - 1);
        src = 1 - src;
    }
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) ignore(hipGraphDestroy(g));
        return fail(LBM_E_HIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&b->graph[parity], g, nullptr, nullptr, 0);
    ignore(hipGraphDestroy(g));
    if (e != hipSuccess) {
        b->graph[parity] = nullptr;
        return fail(LBM_E_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    return LBM_OK;
}

lbm_status apply_launch(lbm_batch* b, const lbm_batch_launch& l)
{
    if (l.block != 128 && l.block != 256 && l.block != 512 && l.block != 1024)
        return fail(LBM_E_INVAL, "batch block %d not one of 128, 256, 512, 1024", l.block);
    if (l.graph_steps < 2 || (l.graph_steps & 1)) return fail(LBM_E_INVAL, "graph_steps %d must be even and >= 2",
                                                              l.graph_steps);
    if (l.blocks_per_cu < 0 || l.blocks_per_cu > 64) return fail(LBM_E_INVAL, "blocks_per_cu %d out of range",
                                                                 l.blocks_per_cu);
    const uint32_t links = max_links_per_tile(b, l.block);
    if (lbm::step_lds_bytes(b->fp32, links) > lbm::kMaxLds)
        return fail(LBM_E_INVAL, "block %d would stage %u wall links, more than the LDS limit", l.block, links);
    LBM_HIP_TRY(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    b->launch = l;
    b->lds_links = links;
    return rebuild_tiles(b);
}

// Copies instance i's state (its plane segments and link range) from buffer `from` to `to`.
lbm_status move_state(lbm_batch* b, int32_t i, int from, int to)
{
    const size_t es = b->esize();
    for (int p = 0; p < 9; ++p) {
        const size_t o = (size_t(p) * b->ps + b->off[i]) * es;
        LBM_HIP_TRY(hipMemcpyAsync(static_cast<char*>(b->d_buf[to]) + o, static_cast<char*>(b->d_buf[from]) + o,
                                   size_t(b->pr[i].n) * es, hipMemcpyDeviceToDevice, b->stream));
    }
    if (b->pr[i].n_links > 0)
        LBM_HIP_TRY(hipMemcpyAsync(static_cast<char*>(b->d_link[to]) + size_t(b->link_off[i]) * es,
                                   static_cast<char*>(b->d_link[from]) + size_t(b->link_off[i]) * es,
                                   size_t(b->pr[i].n_links) * es, hipMemcpyDeviceToDevice, b->stream));
    return LBM_OK;
}

lbm_status step_eager(lbm_batch* b, bool write_u)
{
    const hipError_t e = launch_one(b, b->cur, 1 - b->cur, write_u);
    if (e != hipSuccess) return fail(LBM_E_HIP, "batch step launch: %s", hipGetErrorString(e));
    b->cur = 1 - b->cur;
    return LBM_OK;
}

lbm::Geo instance_geo(const lbm_batch* b, int32_t i)
{
    const lbm::Prepared& p = b->pr[i];
    return lbm::Geo{b->d_flags + b->off[i], b->d_chunk + b->off[i] / lbm::kChunk, p.n, p.nx, p.ny, p.nchunks, b->ps};
}

int state_buffer(const lbm_batch* b, int32_t i) { return b->active[i] ? b->cur : b->inst_cur[i]; }

template <typename T>
std::vector<lbm::BatchInst<T>> inst_table(const lbm_batch* b)
{
    std::vector<lbm::BatchInst<T>> t(size_t(b->n_inst));
    for (int32_t i = 0; i < b->n_inst; ++i) {
        t[i].off = b->off[i];
        t[i].n = b->pr[i].n;
        t[i].nx = b->pr[i].nx;
        t[i].ny = b->pr[i].ny;
        t[i].ph = lbm::make_phys<T>(b->pr[i].p, b->pr[i].g);
    }
    return t;
}

// Uploads instance i's record of the device instance table (its physical constants).
lbm_status upload_inst(lbm_batch* b, int32_t i)
{
    hipError_t e;
    if (b->fp32) {
        const auto t = inst_table<float>(b);
        e = hipMemcpyAsync(static_cast<lbm::BatchInst<float>*>(b->d_inst) + i, &t[size_t(i)],
                           sizeof(lbm::BatchInst<float>), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    } else {
        const auto t = inst_table<double>(b);
        e = hipMemcpyAsync(static_cast<lbm::BatchInst<double>*>(b->d_inst) + i, &t[size_t(i)],
                           sizeof(lbm::BatchInst<double>), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    }
    if (e != hipSuccess) return fail(LBM_E_HIP, "instance table upload: %s", hipGetErrorString(e));
    return LBM_OK;
}

// Rest state of instance i in both buffers (its plane segments, link range and u record).
lbm_status zero_instance(lbm_batch* b, int32_t i)
{
    const size_t es = b->esize();
    for (int buf = 0; buf < 2; ++buf) {
        for (int p = 0; p < 9; ++p)
            LBM_HIP_TRY(lbm::launch_fill_zero(static_cast<char*>(b->d_buf[buf]) + (size_t(p) * b->ps + b->off[i]) * es,
                                              size_t(b->pr[i].n) * es, b->stream));
        if (b->pr[i].n_links > 0)
            LBM_HIP_TRY(lbm::launch_fill_zero(static_cast<char*>(b->d_link[buf]) + size_t(b->link_off[i]) * es,
                                              size_t(b->pr[i].n_links) * es, b->stream));
    }
    for (int c = 0; c < 2; ++c)
        LBM_HIP_TRY(lbm::launch_fill_zero(b->d_uprev + size_t(c) * b->ps + b->off[i], sizeof(double) * b->pr[i].n,
                                          b->stream));
    return LBM_OK;
}

std::string arch_name(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string s = prop.gcnArchName;
    const size_t c = s.find(':');
    return c == std::string::npos ? s : s.substr(0, c);
}

}  // namespace

extern "C" {

lbm_status lbm_batch_create(int32_t n_inst, const lbm_params* params, const uint8_t* const* solids,
                            const lbm_link* const* links, const int64_t* n_links, void* stream, lbm_batch** out)
{
    if (!out) return fail(LBM_E_INVAL, "null output pointer");
    *out = nullptr;
    if (n_inst <= 0 || !params || !solids || !links || !n_links) return fail(LBM_E_INVAL, "empty or null batch input");
    lbm_batch* b = new lbm_batch();
    b->n_inst = n_inst;
    b->pr.resize(size_t(n_inst));
    b->fp32 = params[0].precision == LBM_FP32_SHIFTED;
    b->node = params[0].diffuse == LBM_DIFFUSE_NODE;
    uint64_t sites = 0;
    int64_t nl_total = 0;
    for (int32_t i = 0; i < n_inst; ++i) {
        if (params[i].precision != params[0].precision || params[i].diffuse != params[0].diffuse) {
            release(b);
            return fail(LBM_E_INVAL, "instance %d: precision and diffuse reading must match instance 0", i);
        }
        lbm_status st = lbm::prepare(&params[i], solids[i], links[i], n_links[i], b->pr[i]);
        if (st != LBM_OK) {
            std::string msg = lbm_last_error();
            release(b);
            return fail(st, "instance %d: %s", i, msg.c_str());
        }
        b->off.push_back(uint32_t(sites));
        b->link_off.push_back(nl_total);
        sites += (uint64_t(b->pr[i].n) + kPad - 1) / kPad * kPad;
        nl_total += b->pr[i].n_links;
        if (sites >= (uint64_t(1) << 31)) {
            release(b);
            return fail(LBM_E_INVAL, "batch exceeds 2^31 sites");
        }
        if (nl_total > INT32_MAX) {  // global link offsets in the int32 chunk table
            release(b);
            return fail(LBM_E_INVAL, "batch exceeds 2^31 - 1 wall links");
        }
    }
    b->ps = uint32_t(sites);
    b->total_links = nl_total;
    // global flags and chunk table over the padded site space
    std::vector<uint8_t> flags(b->ps, uint8_t(lbm::kSolid));
    const uint32_t nchunks = b->ps / lbm::kChunk;
    b->chunk.assign(nchunks + 1, 0);
    for (int32_t i = 0; i < n_inst; ++i) {
        const lbm::Prepared& p = b->pr[i];
        std::copy(p.flags.begin(), p.flags.end(), flags.begin() + b->off[i]);
        const uint32_t c0 = b->off[i] / lbm::kChunk;
        const uint32_t c1 = (i + 1 < n_inst) ? b->off[i + 1] / lbm::kChunk : nchunks;
        for (uint32_t c = c0; c < c1; ++c) {
            const uint32_t lc = c - c0;
            b->chunk[c] = int32_t(b->link_off[i] + (lc <= p.nchunks ? p.chunk[lc] : p.chunk[p.nchunks]));
        }
    }
    b->chunk[nchunks] = int32_t(nl_total);
    b->active.assign(size_t(n_inst), 1);
    b->inst_cur.assign(size_t(n_inst), 0);
    b->steps.assign(size_t(n_inst), 0);
    b->uvalid.assign(size_t(n_inst), 0);
    b->last_res.assign(size_t(n_inst), HUGE_VAL);
    b->last_mass.assign(size_t(n_inst), 0.0);
    b->n_clamped.assign(size_t(n_inst), 0);
    b->n_nonconvex.assign(size_t(n_inst), 0);
    for (int32_t i = 0; i < n_inst; ++i) b->tile_capacity += (b->pr[i].n + 127) / 128;

    // --- device ---
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return fail(LBM_E_HIP, "no HIP device available");
    }
    b->on_device = true;
    if (hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess)
        b->n_cu = 256;
    if (stream) {
        b->stream = static_cast<hipStream_t>(stream);
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            release(b);
            return fail(LBM_E_HIP, "stream creation failed");
        }
        b->own_stream = true;
    }
    const size_t nl = size_t(b->link_stride());
    const size_t inst_bytes = b->fp32 ? sizeof(lbm::BatchInst<float>) : sizeof(lbm::BatchInst<double>);
    auto alloc = [&](void** ptr, size_t bytes) -> bool { return hipMalloc(ptr, bytes) == hipSuccess; };
    bool ok = alloc(reinterpret_cast<void**>(&b->d_flags), b->ps) &&
              alloc(reinterpret_cast<void**>(&b->d_chunk), sizeof(int32_t) * (nchunks + 1)) &&
              alloc(reinterpret_cast<void**>(&b->d_coef64), sizeof(double) * 8 * nl) &&
              (!b->fp32 || alloc(reinterpret_cast<void**>(&b->d_coef32), sizeof(float) * 5 * nl)) &&
              alloc(&b->d_buf[0], b->pop_bytes()) && alloc(&b->d_buf[1], b->pop_bytes()) &&
              alloc(&b->d_link[0], b->link_bytes()) && alloc(&b->d_link[1], b->link_bytes()) &&
              alloc(reinterpret_cast<void**>(&b->d_uprev), sizeof(double) * 2 * b->ps) &&
              alloc(&b->d_inst, inst_bytes * size_t(n_inst)) &&
              alloc(reinterpret_cast<void**>(&b->d_tiles), sizeof(lbm::TileRef) * b->tile_capacity) &&
              alloc(reinterpret_cast<void**>(&b->d_n_active), sizeof(uint32_t)) &&
              alloc(reinterpret_cast<void**>(&b->d_tile_begin), sizeof(uint32_t) * (size_t(n_inst) + 1)) &&
              alloc(reinterpret_cast<void**>(&b->d_partial), sizeof(double) * 3 * b->tile_capacity) &&
              alloc(reinterpret_cast<void**>(&b->d_result), sizeof(double) * 3 * size_t(n_inst)) &&
              hipHostMalloc(reinterpret_cast<void**>(&b->h_result), sizeof(double) * 3 * size_t(n_inst),
                            hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        release(b);
        return fail(LBM_E_NOMEM, "device allocation failed for a batch of %u sites", b->ps);
    }
    hipError_t he = hipMemcpyAsync(b->d_flags, flags.data(), b->ps, hipMemcpyHostToDevice, b->stream);
    if (he == hipSuccess)
        he = hipMemcpyAsync(b->d_chunk, b->chunk.data(), sizeof(int32_t) * (nchunks + 1), hipMemcpyHostToDevice,
                            b->stream);
    if (he == hipSuccess) {
        if (b->fp32) {
            auto t = inst_table<float>(b);
            he = hipMemcpyAsync(b->d_inst, t.data(), inst_bytes * t.size(), hipMemcpyHostToDevice, b->stream);
            if (he == hipSuccess) he = hipStreamSynchronize(b->stream);
        } else {
            auto t = inst_table<double>(b);
            he = hipMemcpyAsync(b->d_inst, t.data(), inst_bytes * t.size(), hipMemcpyHostToDevice, b->stream);
            if (he == hipSuccess) he = hipStreamSynchronize(b->stream);
        }
    }
    if (he != hipSuccess) {
        release(b);
        return fail(LBM_E_HIP, "batch upload failed: %s", hipGetErrorString(he));
    }
    for (int32_t i = 0; i < n_inst; ++i) {
        lbm_status st = lbm::precompute_links(b->pr[i], b->d_coef64, b->fp32 ? b->d_coef32 : nullptr,
                                              b->link_stride(), b->link_off[i], b->stream, b->n_clamped[i],
                                              b->n_nonconvex[i]);
        if (st != LBM_OK) {
            std::string msg = lbm_last_error();
            release(b);
            return fail(st, "instance %d: %s", i, msg.c_str());
        }
    }
    lbm_batch_launch l{256, 10, 4, 0};
    lbm_status st = apply_launch(b, l);
    if (st == LBM_OK) st = lbm_batch_init_rest(b);
    if (st != LBM_OK) {
        release(b);
        return st;
    }
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_destroy(lbm_batch* b)
{
    release(b);
    return LBM_OK;
}

lbm_status lbm_batch_info(const lbm_batch* b, int32_t i, lbm_info* info)
{
    if (!b || !info || i < 0 || i >= b->n_inst) return fail(LBM_E_INVAL, "bad batch or instance");
    const lbm::Prepared& p = b->pr[i];
    std::memset(info, 0, sizeof *info);
    info->tau_s = p.g.tau_s;
    info->tau_q = p.g.tau_q;
    info->E = p.g.E;
    info->E_max = p.g.E_max;
    info->L1 = p.g.L1;
    info->L2 = p.g.L2;
    info->nu = (p.g.tau_s - 0.5) / 3.0;
    info->n_sites = p.n;
    info->n_fluid = p.n_fluid;
    info->n_links = p.n_links;
    info->n_clamped = b->n_clamped[i];
    info->n_nonconvex = b->n_nonconvex[i];
    info->precision = p.p.precision;
    const int64_t sz = int64_t(b->esize());
    info->bytes_per_step = 18 * sz * p.n_fluid + (5 + 5 * sz) * p.n_links + int64_t(p.n);
    info->steps = b->steps[i];
    return LBM_OK;
}

lbm_status lbm_batch_init_rest(lbm_batch* b)
{
    if (!b) return fail(LBM_E_INVAL, "null batch");
    DeviceGuard g(b->device);
    LBM_HIP_TRY(lbm::launch_fill_zero(b->d_buf[0], b->pop_bytes(), b->stream));
    LBM_HIP_TRY(lbm::launch_fill_zero(b->d_buf[1], b->pop_bytes(), b->stream));
    LBM_HIP_TRY(lbm::launch_fill_zero(b->d_link[0], b->link_bytes(), b->stream));
    LBM_HIP_TRY(lbm::launch_fill_zero(b->d_link[1], b->link_bytes(), b->stream));
    LBM_HIP_TRY(lbm::launch_fill_zero(b->d_uprev, sizeof(double) * 2 * b->ps, b->stream));
    b->cur = 0;
    std::fill(b->active.begin(), b->active.end(), 1);
    std::fill(b->inst_cur.begin(), b->inst_cur.end(), 0);
    std::fill(b->steps.begin(), b->steps.end(), 0);
    std::fill(b->uvalid.begin(), b->uvalid.end(), 0);
    std::fill(b->last_res.begin(), b->last_res.end(), HUGE_VAL);
    return rebuild_tiles(b);
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps)
{
    if (!b) return fail(LBM_E_INVAL, "null batch");
    if (nsteps < 0) return fail(LBM_E_INVAL, "negative step count");
    if (nsteps == 0 || b->n_active_tiles == 0) return LBM_OK;
    DeviceGuard g(b->device);
    const int64_t G = b->launch.graph_steps;
    const int64_t q = nsteps / G, r = nsteps % G;
    for (int64_t k = 0; k < q; ++k) {
        if (!b->graph[b->cur]) {
            lbm_status st = capture(b, b->cur);
            if (st != LBM_OK) return st;
        }
        LBM_HIP_TRY(hipGraphLaunch(b->graph[b->cur], b->stream));
    }
    for (int64_t k = 0; k < r; ++k) {
        lbm_status st = step_eager(b, k == r - 1);
        if (st != LBM_OK) return st;
    }
    for (int32_t i = 0; i < b->n_inst; ++i)
        if (b->active[i]) {
            b->steps[i] += nsteps;
            b->uvalid[i] = 1;
        }
    return LBM_OK;
}

lbm_status lbm_batch_set_active(lbm_batch* b, const uint8_t* act)
{
    if (!b || !act) return fail(LBM_E_INVAL, "null argument");
    DeviceGuard g(b->device);
    bool changed = false;
    for (int32_t i = 0; i < b->n_inst; ++i) {
        const uint8_t want = act[i] ? 1 : 0;
        if (want == b->active[i]) continue;
        changed = true;
        if (!want) {
            b->inst_cur[i] = b->cur;
        } else if (b->inst_cur[i] != b->cur) {
            lbm_status st = move_state(b, i, b->inst_cur[i], b->cur);
            if (st != LBM_OK) return st;
        }
        b->active[i] = want;
    }
    return changed ? rebuild_tiles(b) : LBM_OK;
}

lbm_status lbm_batch_residuals(lbm_batch* b, double* residual, double* mass)
{
    if (!b || !residual || !mass) return fail(LBM_E_INVAL, "null argument");
    DeviceGuard g(b->device);
    const uint32_t n_act = uint32_t(b->active_list.size());
    if (n_act > 0) {
        const uint32_t grid = grid_of(b);
        if (b->fp32) {
            lbm::BatchReduceArgs<float> a{b->d_flags, b->d_chunk, static_cast<const float*>(b->d_buf[b->cur]),
                                          static_cast<const float*>(b->d_link[b->cur]), b->d_uprev,
                                          b->d_uprev + b->ps, static_cast<const lbm::BatchInst<float>*>(b->d_inst),
                                          b->d_tiles, b->d_n_active, b->d_partial, b->ps};
            LBM_HIP_TRY(lbm::launch_residual_batch_f32(a, b->launch.block, grid, b->d_tile_begin, n_act, b->d_result,
                                                       b->stream));
        } else {
            lbm::BatchReduceArgs<double> a{b->d_flags, b->d_chunk, static_cast<const double*>(b->d_buf[b->cur]),
                                           static_cast<const double*>(b->d_link[b->cur]), b->d_uprev,
                                           b->d_uprev + b->ps, static_cast<const lbm::BatchInst<double>*>(b->d_inst),
                                           b->d_tiles, b->d_n_active, b->d_partial, b->ps};
            LBM_HIP_TRY(lbm::launch_residual_batch_f64(a, b->launch.block, grid, b->d_tile_begin, n_act, b->d_result,
                                                       b->stream));
        }
        LBM_HIP_TRY(hipMemcpyAsync(b->h_result, b->d_result, sizeof(double) * 3 * n_act, hipMemcpyDeviceToHost,
                                   b->stream));
        LBM_HIP_TRY(hipStreamSynchronize(b->stream));
    }
    bool bad = false;
    for (uint32_t k = 0; k < n_act; ++k) {
        const int32_t i = b->active_list[k];
        const double s_du = b->h_result[3 * k], s_u = b->h_result[3 * k + 1], s_dr = b->h_result[3 * k + 2];
        b->last_mass[i] = double(b->pr[i].n_fluid) * b->pr[i].p.rho0 + s_dr;
        b->last_res[i] = b->uvalid[i] ? std::sqrt(s_du / s_u) : HUGE_VAL;
        if (!std::isfinite(s_du) || !std::isfinite(s_u) || !std::isfinite(s_dr)) {
            b->last_res[i] = std::nan("");
            bad = true;
        }
    }
    for (int32_t i = 0; i < b->n_inst; ++i) {
        residual[i] = b->last_res[i];
        mass[i] = b->last_mass[i];
    }
    return bad ? fail(LBM_E_UNSTABLE, "an active batch instance is not finite") : LBM_OK;
}

lbm_status lbm_batch_moments(lbm_batch* b, int32_t i, double* rho, double* ux, double* uy, int32_t device_ptrs)
{
    if (!b || !rho || !ux || !uy || i < 0 || i >= b->n_inst) return fail(LBM_E_INVAL, "bad argument");
    DeviceGuard g(b->device);
    const lbm::Prepared& p = b->pr[i];
    const int buf = state_buffer(b, i);
    const void* pop = static_cast<const char*>(b->d_buf[buf]) + size_t(b->off[i]) * b->esize();
    double *r = rho, *u = ux, *v = uy;
    double* stage = nullptr;
    if (!device_ptrs) {
        LBM_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&stage), sizeof(double) * 3 * p.n));
        r = stage;
        u = stage + p.n;
        v = stage + 2 * size_t(p.n);
    }
    hipError_t e = lbm::launch_moments(b->fp32, instance_geo(b, i), pop, b->d_link[buf], r, u, v, p.p.rho0, p.p.ax,
                                       p.p.ay, b->stream);
    if (!device_ptrs) {
        if (e == hipSuccess) e = hipMemcpyAsync(rho, r, sizeof(double) * p.n, hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(ux, u, sizeof(double) * p.n, hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(uy, v, sizeof(double) * p.n, hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        ignore(hipFree(stage));
    }
    if (e != hipSuccess) return fail(LBM_E_HIP, "batch moments: %s", hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_batch_solve(lbm_batch* b, double tol, int64_t check_every, int64_t max_steps, int32_t* status,
                           int64_t* steps_out, double* residual_out)
{
    if (!b) return fail(LBM_E_INVAL, "null batch");
    if (check_every < 2 || (check_every & 1)) return fail(LBM_E_INVAL, "check_every must be even and >= 2");
    const int32_t n = b->n_inst;
    const size_t nn = static_cast<size_t>(n);
    std::vector<int32_t> st(nn, LBM_RUNNING);
    std::vector<std::vector<double>> hist(nn);
    std::vector<double> res(nn), mass(nn);
    for (int32_t i = 0; i < n; ++i)
        if (!b->active[i]) st[i] = LBM_CAPPED;  // retired before the solve: left as they are
    while (!b->active_list.empty()) {
        lbm_status s = lbm_batch_step(b, check_every);
        if (s != LBM_OK) return s;
        s = lbm_batch_residuals(b, res.data(), mass.data());
        if (s != LBM_OK && s != LBM_E_UNSTABLE) return s;
        std::vector<uint8_t> act(b->active);
        for (int32_t i : b->active_list) {
            const double R = res[i];
            hist[i].push_back(R);
            if (!std::isfinite(R) || !std::isfinite(mass[i])) st[i] = LBM_DIVERGED;
            else if (R <= tol) st[i] = LBM_CONVERGED;
            else if (b->steps[i] >= max_steps) st[i] = LBM_CAPPED;
            else if (hist[i].size() > size_t(kFloorWindow) && R < kFloorBelow &&
                     R > kFloorRatio * hist[i][hist[i].size() - 1 - kFloorWindow])
                st[i] = LBM_FLOOR;
            if (st[i] != LBM_RUNNING) act[i] = 0;
        }
        s = lbm_batch_set_active(b, act.data());
        if (s != LBM_OK) return s;
    }
    for (int32_t i = 0; i < n; ++i) {
        if (status) status[i] = st[i];
        if (steps_out) steps_out[i] = b->steps[i];
        if (residual_out) residual_out[i] = b->last_res[i];
    }
    return LBM_OK;
}

lbm_status lbm_batch_set_params(lbm_batch* b, int32_t i, const lbm_params* p)
{
    if (!b || !p || i < 0 || i >= b->n_inst) return fail(LBM_E_INVAL, "bad batch, instance or params");
    const lbm::Prepared& old = b->pr[i];
    if (p->nx != old.p.nx || p->ny != old.p.ny || p->periodic_x != old.p.periodic_x ||
        p->periodic_y != old.p.periodic_y)
        return fail(LBM_E_INVAL, "instance %d: lattice size and periodicity cannot change", i);
    if (p->precision != old.p.precision || p->diffuse != old.p.diffuse)
        return fail(LBM_E_INVAL, "instance %d: precision and diffuse reading are fixed per batch", i);
    DeviceGuard g(b->device);
    lbm::Prepared np = old;
    np.p = *p;
    lbm_status st = lbm::check_params(np.p, np.g);
    if (st != LBM_OK) return st;
    LBM_HIP_TRY(hipStreamSynchronize(b->stream));
    int32_t ncl = 0, nnc = 0;
    st = lbm::precompute_links(np, b->d_coef64, b->fp32 ? b->d_coef32 : nullptr, b->link_stride(), b->link_off[i],
                               b->stream, ncl, nnc);
    if (st != LBM_OK) {
        // put the previous coefficients back before reporting
        const std::string msg = lbm_last_error();
        int32_t a = 0, c = 0;
        if (lbm::precompute_links(old, b->d_coef64, b->fp32 ? b->d_coef32 : nullptr, b->link_stride(),
                                  b->link_off[i], b->stream, a, c) != LBM_OK)
            return fail(LBM_E_HIP, "instance %d: restoring the previous coefficients failed after: %s", i,
                        msg.c_str());
        return fail(st, "instance %d: %s", i, msg.c_str());
    }
    b->pr[i] = std::move(np);
    b->n_clamped[i] = ncl;
    b->n_nonconvex[i] = nnc;
    st = upload_inst(b, i);
    if (st == LBM_OK) st = zero_instance(b, i);
    if (st != LBM_OK) return st;
    b->inst_cur[i] = b->cur;
    b->steps[i] = 0;
    b->uvalid[i] = 0;
    b->last_res[i] = HUGE_VAL;
    b->last_mass[i] = 0.0;
    if (!b->active[i]) {
        b->active[i] = 1;
        return rebuild_tiles(b);
    }
    return LBM_OK;
}

lbm_status lbm_batch_solve_fallback(lbm_batch* b, double tol, int64_t check_every, int64_t max_steps, int32_t* status,
                                    int64_t* steps_out, double* residual_out, uint8_t* fell_back)
{
    if (!b) return fail(LBM_E_INVAL, "null batch");
    const size_t nn = size_t(b->n_inst);
    std::vector<int32_t> st(nn);
    std::vector<int64_t> steps(nn);
    std::vector<double> res(nn);
    lbm_status s = lbm_batch_solve(b, tol, check_every, max_steps, st.data(), steps.data(), res.data());
    if (s != LBM_OK) return s;
    std::vector<uint8_t> again(nn, 0);
    bool any = false;
    for (int32_t i = 0; i < b->n_inst; ++i)
        if (st[i] == LBM_DIVERGED && b->pr[i].p.l_mode == LBM_L_PAPER) {
            lbm_params p = b->pr[i].p;
            p.l_mode = LBM_L_CLAMP_NEG;
            s = lbm_batch_set_params(b, i, &p);
            if (s != LBM_OK) return s;
            again[i] = 1;
            any = true;
        }
    if (any) {
        // only the re-parametrised instances run; the others stay retired with their state
        s = lbm_batch_set_active(b, again.data());
        if (s != LBM_OK) return s;
        std::vector<int32_t> st2(nn);
        std::vector<int64_t> steps2(nn);
        std::vector<double> res2(nn);
        s = lbm_batch_solve(b, tol, check_every, max_steps, st2.data(), steps2.data(), res2.data());
        if (s != LBM_OK) return s;
        for (size_t i = 0; i < nn; ++i)
            if (again[i]) {
                st[i] = st2[i];
                steps[i] = steps2[i];
                res[i] = res2[i];
            }
    }
    for (size_t i = 0; i < nn; ++i) {
        if (status) status[i] = st[i];
        if (steps_out) steps_out[i] = steps[i];
        if (residual_out) residual_out[i] = res[i];
        if (fell_back) fell_back[i] = again[i];
    }
    return LBM_OK;
}

lbm_status lbm_batch_set_launch(lbm_batch* b, const lbm_batch_launch* l)
{
    if (!b || !l) return fail(LBM_E_INVAL, "null argument");
    DeviceGuard g(b->device);
    return apply_launch(b, *l);
}

lbm_status lbm_batch_get_launch(const lbm_batch* b, lbm_batch_launch* l)
{
    if (!b || !l) return fail(LBM_E_INVAL, "null argument");
    *l = b->launch;
    return LBM_OK;
}

lbm_status lbm_batch_tune(lbm_batch* b, const char* cache_path, int32_t trial_steps, lbm_batch_launch* chosen)
{
    if (!b) return fail(LBM_E_INVAL, "null batch");
    if (trial_steps < 2) trial_steps = 2;
    DeviceGuard g(b->device);
    std::ostringstream key;
    uint64_t fluid = 0;
    for (const auto& p : b->pr) fluid += uint64_t(p.n_fluid);
    key << arch_name(b->device) << "/" << (b->fp32 ? "fp32" : "fp64") << "/sites2^"
        << int(std::log2(double(std::max<uint32_t>(b->ps, 1)))) << "/fluid2^" << int(std::log2(double(std::max<uint64_t>(fluid, 1))))
        << "/inst2^" << int(std::log2(double(b->n_inst)));
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string k;
        lbm_batch_launch l{};
        double ms = 0;
        while (in >> k >> l.block >> l.graph_steps >> l.blocks_per_cu >> ms)
            if (k == key.str()) {
                lbm_status st = apply_launch(b, l);
                if (st == LBM_OK) st = lbm_batch_init_rest(b);
                if (st == LBM_OK && chosen) *chosen = b->launch;
                return st;
            }
    }
    hipEvent_t e0, e1;
    LBM_HIP_TRY(hipEventCreate(&e0));
    LBM_HIP_TRY(hipEventCreate(&e1));
    lbm_batch_launch best = b->launch;
    double best_ms = HUGE_VAL;
    // one trial: capture and warm up, then time n steps; any failure ends the tuning with its status
    auto trial = [&](const lbm_batch_launch& l) -> lbm_status {
        if (apply_launch(b, l) != LBM_OK) return LBM_OK;  // shape not usable here (e.g. LDS): skipped
        const int64_t n = (int64_t(trial_steps) + l.graph_steps - 1) / l.graph_steps * l.graph_steps;
        lbm_status st = lbm_batch_step(b, l.graph_steps);
        if (st != LBM_OK) return st;
        LBM_HIP_TRY(hipEventRecord(e0, b->stream));
        st = lbm_batch_step(b, n);
        if (st != LBM_OK) return st;
        LBM_HIP_TRY(hipEventRecord(e1, b->stream));
        LBM_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0;
        LBM_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        const double per = double(ms) / double(n);
        if (per < best_ms) {
            best_ms = per;
            best = l;
        }
        return LBM_OK;
    };
    lbm_status status = LBM_OK;
    for (int blk : {128, 256, 512})
        for (int gs : {2, 10, 50})
            for (int bpc : {0, 2, 4, 8})
                if (status == LBM_OK) status = trial(lbm_batch_launch{blk, gs, bpc, 0});
    ignore(hipEventDestroy(e0));
    ignore(hipEventDestroy(e1));
    if (status != LBM_OK) return status;
    lbm_status st = apply_launch(b, best);
    if (st == LBM_OK) st = lbm_batch_init_rest(b);
    if (st != LBM_OK) return st;
    if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        o << key.str() << " " << best.block << " " << best.graph_steps << " " << best.blocks_per_cu << " " << best_ms
          << "\n";
    }
    if (chosen) *chosen = best;
    return LBM_OK;
}

}  // extern "C"
