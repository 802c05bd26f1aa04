// Internal declarations shared by the C-ABI host code and the HIP kernels of liblbm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

// Site flag byte: 0xFF marks a solid site; otherwise bit (d-1) is set when the neighbour
// x + c_d is solid, i.e. when (x, d) is a wall link.  A fluid site with all eight neighbours
// solid would collide with the solid code and is rejected at creation.
constexpr uint32_t kSolid = 0xFFu;

// Sites are grouped in aligned chunks of one wavefront (64 sites); chunk_base[c] is the number
// of wall links owned by sites < 64 c.  Links are stored sorted by (site, direction), so the
// links of a site, of a wavefront and of a block are contiguous index ranges.
constexpr int kChunk = 64;
constexpr int kFuseTX = 64;  // tile width of the two-step kernel (one chunk)

// Lattice geometry shared by every kernel.  Population plane i starts at element i * ps, with the
// plane stride ps = n rounded up to a whole number of 64-site chunks, so that every plane starts on
// a 128-byte line and a wavefront's 64 sites cover whole lines.
struct Geo {
    const uint8_t* flags;      // n
    const int32_t* chunk_base; // nchunks + 1
    uint32_t n, nx, ny, nchunks;
    uint32_t ps;               // plane stride (elements)
};

// Per-link boundary coefficients in the storage precision, one array each (structure of arrays).
template <typename T>
struct LinkCoef {
    const T* a1;
    const T* a2;
    const T* a3;
    const T* beta;
    const T* kappa;
};

// One time level of the state: nine population planes in pull layout (plane i at site y holds the
// value site y + c_i receives) and, per wall link (x, d), the population opposite(d) that x
// receives from the wall.
template <typename T>
struct Level {
    T* pop;
    T* link;
};

// Arguments of the fused collide-stream-boundary kernel.
template <typename T>
struct StepArgs {
    Geo g;
    Level<T> src, dst;
    LinkCoef<T> coef;
    double* ux_out;            // n, written only when the kernel is asked to record u
    double* uy_out;
    uint32_t lds_links;        // link slots of the LDS staging area (max links of one block)
    T rho0, ax, ay;
    T s_e, s_eps, s_q, s_s;    // relaxation rates 1/tau
    T c_e, c_eps, c_q, c_s;    // 1 - s/2 (forcing weights)
};

// Physical constants of one lattice in the storage precision.
template <typename T>
struct Phys {
    T rho0, ax, ay;
    T s_e, s_eps, s_q, s_s;
    T c_e, c_eps, c_q, c_s;
};

// One instance of a batch: its sites occupy [off, off + n) of the batch's site space (off is a
// multiple of the largest tile), laid out as an nx x ny lattice.
template <typename T>
struct BatchInst {
    uint32_t off, n, nx, ny;
    Phys<T> ph;
};

// One tile of an active instance: `start` is the tile's first site, local to the instance.
struct TileRef {
    uint32_t inst, start;
};

// Arguments of the batched persistent step kernel.
template <typename T>
struct BatchArgs {
    const uint8_t* flags;         // batch site space
    const int32_t* chunk_base;    // per 64-site chunk of the batch site space; global link indices
    Level<T> src, dst;            // planes over the batch site space (stride ps); link arrays global
    LinkCoef<T> coef;             // global link indices
    double* ux_out;               // batch site space
    double* uy_out;
    const BatchInst<T>* inst;
    const TileRef* tiles;         // active tiles, instance by instance
    const uint32_t* n_active;     // number of active tiles (device resident, read at launch)
    uint32_t ps;                  // plane stride of the batch site space
    uint32_t lds_links;           // link slots of the LDS staging area (max links of one tile)
};

// Batched residual: per active tile partial sums, then per active instance a fixed-order sum over
// its tile range [tile_begin[i], tile_begin[i+1]) of the active list.
template <typename T>
struct BatchReduceArgs {
    const uint8_t* flags;
    const int32_t* chunk_base;
    const T* pop;
    const T* link;
    const double* ux_prev;
    const double* uy_prev;
    const BatchInst<T>* inst;
    const TileRef* tiles;
    const uint32_t* n_active;
    double* partial;              // 3 per active tile
    uint32_t ps;
};

struct LinkInput {
    const double* q;
    const double* ubx;
    const double* uby;
    const int32_t* dir;
};

// Global parameters of the prescription needed by the per-link precompute.
struct PrecomputeArgs {
    double tau_s, tau_q, L1, L2, E, sq6pi;
    double r_override, l_override;
    int32_t l_mode, r_mode, diffuse;
    int64_t n_links;
    int64_t row_stride;  // elements between coefficient rows (>= n_links)
};

struct ReduceArgs {
    Geo g;
    const void* pop;
    const void* link;
    const double* ux_prev;
    const double* uy_prev;
    double* partial;  // 3 per block
    double rho0, ax, ay;
};

// Launchers (lbm_kernels.hip).  All are asynchronous on `stream`.
hipError_t launch_precompute(const LinkInput& in, const PrecomputeArgs& a, double* coef64, float* coef32,
                             hipStream_t stream);
// Bytes of LDS one block of `block` threads needs for `max_links` wall links.
size_t step_lds_bytes(bool fp32, uint32_t max_links);
// Two steps per launch on 64 x rows tiles (rows: 4 or 8); a.lds_links must hold the wall links of
// any tile.  Needs nx % 64 == 0 and ny % rows == 0.
size_t step2_lds_bytes(bool fp32, int rows, uint32_t max_links);
hipError_t launch_step2_f64(const StepArgs<double>& a, int rows, bool write_u, bool node_diffuse, hipStream_t stream);
hipError_t launch_step2_f32(const StepArgs<float>& a, int rows, bool write_u, bool node_diffuse, hipStream_t stream);
hipError_t launch_step_f64(const StepArgs<double>& a, int block, bool write_u, bool node_diffuse,
                           hipStream_t stream);
hipError_t launch_step_f32(const StepArgs<float>& a, int block, bool write_u, bool node_diffuse,
                           hipStream_t stream);
// Batched persistent step over the active tile list with a grid of `grid` blocks of `block` threads.
hipError_t launch_step_batch_f64(const BatchArgs<double>& a, int block, uint32_t grid, bool write_u,
                                 bool node_diffuse, hipStream_t stream);
hipError_t launch_step_batch_f32(const BatchArgs<float>& a, int block, uint32_t grid, bool write_u,
                                 bool node_diffuse, hipStream_t stream);
// Per-active-instance sums (|du|^2, |u|^2, sum drho) into out[3 * i] for the active instances
// i = 0 .. n_inst_active-1, whose tiles are tile_begin[i] .. tile_begin[i+1]-1 of the active list.
hipError_t launch_residual_batch_f64(const BatchReduceArgs<double>& a, int block, uint32_t grid,
                                     const uint32_t* tile_begin, uint32_t n_inst_active, double* out,
                                     hipStream_t stream);
hipError_t launch_residual_batch_f32(const BatchReduceArgs<float>& a, int block, uint32_t grid,
                                     const uint32_t* tile_begin, uint32_t n_inst_active, double* out,
                                     hipStream_t stream);
hipError_t launch_fill_zero(void* ptr, uint64_t bytes, hipStream_t stream);
// Copies bytes (a multiple of 16; both pointers 16-byte aligned) from src to dst.
hipError_t launch_stream_copy(void* dst, const void* src, uint64_t bytes, hipStream_t stream);
// f = f^eq(rho, u - a/2) at fluid sites; with neq_tau = tau_s > 0 plus the first-order
// non-equilibrium of the stress moments from the fluid-neighbour differences of u.
hipError_t launch_init_fields(bool fp32, const Geo& g, void* pop, void* link, const double* rho, const double* ux,
                              const double* uy, double rho0, double ax, double ay, double neq_tau, hipStream_t stream);
hipError_t launch_moments(bool fp32, const Geo& g, const void* pop, const void* link, double* rho, double* ux,
                          double* uy, double rho0, double ax, double ay, hipStream_t stream);
// Residual partial sums (|du|^2, |u|^2, sum of density deviations) and the fixed-order final
// reduction into out[0..2].
hipError_t launch_residual(bool fp32, const ReduceArgs& a, double* out, hipStream_t stream);
uint32_t residual_blocks(uint32_t n);

}  // namespace lbm
