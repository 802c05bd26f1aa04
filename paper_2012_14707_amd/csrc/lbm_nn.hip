// Learned warm start: a convolutional encoder-decoder that maps the problem statement (mask,
// distance ratios, Kn, force direction) to an initial (u, rho) for the lattice solver, trained on
// steady fields that the solver computes.  Hand-written for gfx950: convolutions are implicit GEMMs
// on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16) with fp32 accumulation; activations are
// NHWC bf16; master weights, gradients and Adam state are fp32.
//
// Network (levels L, base channels C): encoder level l has C 2^l channels and two 3x3
// convolutions with ReLU; levels are joined by 2x2 average pooling.  Decoder level l (L-2 .. 0)
// upsamples the level below (nearest), concatenates the encoder output of level l, and applies two
// 3x3 convolutions with ReLU.  A 1x1 convolution gives the outputs.  The encoder output of level l
// is written straight into the second channel slice of decoder level l's concatenation buffer, so
// the skip connection costs no copy; where the halo-tile kernels run, the pooling and the output 1x1
// convolution are done in the output stage of the convolution before them, and the decoder's first
// convolution (forward and weight gradient) reads the upsampled channels straight from the level
// below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

#include "lbm.h"
#include "lbm_host.hpp"
#include "lbm_internal.hpp"

using lbm::DeviceGuard;
using lbm::fail;
using lbm::ignore;

namespace lbm {
namespace nn {

typedef __bf16 bf16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(4))) float f4;

// ------------------------------------------------------------------------ matrix-core GEMMs

constexpr int TM = 64, TN = 64, TK = 32;

// A channel slice of an NHWC bf16 tensor: element (pixel p, channel c) at p * cs + co + c.
struct Slice {
    bf16* p;
    int cs, co;
};
struct CSlice {
    const bf16* p;
    int cs, co;
};

struct ConvArgs {
    CSlice x;           // input, Cin channels
    const bf16* w;      // [taps][Cout][Cin], Cin contiguous
    const float* bias;  // [Cout] or null
    Slice y;            // bf16 output (y.p null: none)
    float* yf;          // fp32 output [pixels][Cout] (null: none)
    int N, H, W, Cin, Cout, relu;
    int periodic;       // 1: rows and columns wrap around; 0: zero padding
    float* part;        // split K: fp32 partial sums [splits][pixels][Cout] (null: no split)
    int kper;           // split K: K range of one split (a multiple of TK)
    Slice pool;         // 2x2 mean of the bf16 output at H/2 x W/2 (p null: none; halo-tile kernel only)
    // a 1x1 convolution of the bf16 output (all Cout = 32 channels) into y1, fp32 [pixels][c1]
    // (w1 [c1][32], b1 [c1] or null; w1 null: none; 8 x 32 x 32 halo tiles only)
    const bf16* w1;
    const float* b1;
    float* y1;
    int c1;
    // input channels [0, cup) are the nearest 2x upsampling of up (an H/2 x W/2 image; p null:
    // none; halo-tile kernel only); channels >= cup are read from x
    CSlice up;
    int cup;
};

__device__ __forceinline__ void decompose(int p, int H, int W, int& n, int& y, int& x)
{
    n = p / (H * W);
    const int r = p - n * H * W;
    y = r / W;
    x = r - y * W;
}

// Zeros: the source of the operand chunks that lie outside the image (zero padding), past the end
// of K or past the last pixel or output channel, for the direct-to-LDS loads below.  Such a chunk's
// address is this buffer plus the chunk's channel offset, so it must hold the widest input (the
// largest concatenation the network configuration allows is 12288 channels).
constexpr int kZeroElems = 12288 + 64;
__device__ __align__(16) bf16 g_zero[kZeroElems] = {};

// LDS slot of 16-byte K group q of operand row r in a stage: rows of four groups (64 bytes), the
// group index XOR-swizzled by row so that the 16-byte reads of the MFMA operands (16 consecutive
// rows, one group) fall in distinct banks.
__device__ __forceinline__ int conv_slot(int r, int q) { return r * 4 + (q ^ (((r >> 1) ^ (r >> 3)) & 3)); }

// out[p][co] = act(bias[co] + sum_{tap, ci} x[p + off(tap)][ci] w[tap][co][ci]), with zero padding
// or periodic wrap-around at the image edges.
// One block of four waves computes a BM-pixel x BN-channel tile (the launcher picks the largest of
// 128 x 64, 128 x 32, 64 x 64, 64 x 32 that still gives enough blocks to fill the chip); the waves
// form a WGM x WGN grid and each multiplies a (BM / WGM) x (BN / WGN) part with 16x16x32 MFMAs.  K
// runs over (tap, ci) in steps of TK; Cin is a multiple of 8, so every 8-wide K group lies in one tap
// and is one 16-byte chunk.  NS-stage pipeline: the operand chunks go from global memory straight
// into LDS (16-byte direct loads, no registers), NS - 1 K steps ahead of the multiply, with one
// barrier per K step.  Thread t loads, for each K step, the 16-byte group q(t) of operand rows
// t / 4 + 64 j, whose LDS slots are exactly the 16-byte positions 16 (t + 256 j) that the direct
// load of its wave writes (lane order).  The load addresses advance incrementally with K; the
// per-step integer work is a few adds (a division per step made the kernel bound by vector issue,
// with only 4-8 MFMAs per wave per step).
template <int TAPS, int BM, int BN, int NS>
__global__ void __launch_bounds__(256) k_conv_fwd(const ConvArgs a)
{
    constexpr int WGN = BN >= 64 ? 2 : 1, WGM = 4 / WGN;
    constexpr int MI = BM / WGM / 16, NJ = BN / WGN / 16;
    constexpr int AJ = BM / 64;                   // A rows per thread per K step
    constexpr int BT = BN * 4;                    // threads that load a B group (BN * 4 <= 256)
    static_assert(BT <= 256 && BT % 64 == 0, "B groups fill whole waves");
    extern __shared__ __align__(16) unsigned char smem[];
    bf16* As = reinterpret_cast<bf16*>(smem);                 // [NS][BM * 32]
    bf16* Bs = As + NS * BM * 32;                              // [NS][BN * 32]
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int P = a.N * a.H * a.W;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int kb = a.part ? blockIdx.z * a.kper : 0;
    const int K = a.part ? min(TAPS * a.Cin, kb + a.kper) : TAPS * a.Cin;
    const int nsteps = (K - kb + TK - 1) / TK;
    // this thread's K group (swizzled as the LDS slot it fills) and operand rows
    const int q = (tid & 3) ^ (((tid >> 3) ^ (tid >> 5)) & 3);
    int pn[AJ], py[AJ], px[AJ];
    bool pin[AJ];
#pragma unroll
    for (int j = 0; j < AJ; ++j) {
        const int p = m0 + tid / 4 + 64 * j;
        pin[j] = p < P;
        pn[j] = py[j] = px[j] = 0;
        if (pin[j]) decompose(p, a.H, a.W, pn[j], py[j], px[j]);
    }
    const int co = n0 + tid / 4;
    const bool b_loader = tid < BT;  // wave-uniform (BT is a multiple of 64)
    // The K position of this thread's group walks forward by TK per step.  Each operand row has a
    // base pointer for the current tap (into the zero buffer where the row lies outside the image or
    // the tap is past the last one, which also covers the end of K), and a step's chunk is that base
    // plus the channel offset ci; (tap, ci) advance by adds, and the bases change only every Cin / TK
    // steps.  A division or a bounds test per step made the kernel bound by vector issue.
    int tap = (kb + q * 8) / a.Cin, ci = kb + q * 8 - tap * a.Cin;
    const bf16* zero = g_zero;  // (the lambdas below take the pointer, not the device variable)
    const bf16* abase[AJ];
    const bf16* bbase = zero;
    auto set_tap = [&](int t) __attribute__((always_inline)) {
        const int dy = (TAPS == 9 ? t / 3 - 1 : 0), dx = (TAPS == 9 ? t % 3 - 1 : 0);
#pragma unroll
        for (int j = 0; j < AJ; ++j) {
            int yy = py[j] + dy, xx = px[j] + dx;
            if (a.periodic) {
                yy = yy < 0 ? yy + a.H : (yy >= a.H ? yy - a.H : yy);
                xx = xx < 0 ? xx + a.W : (xx >= a.W ? xx - a.W : xx);
            }
            const bool in = t < TAPS && pin[j] && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
            abase[j] = in ? a.x.p + long((pn[j] * a.H + yy) * a.W + xx) * a.x.cs + a.x.co : zero;
        }
        bbase = (t < TAPS && co < a.Cout) ? a.w + long(t * a.Cout + co) * a.Cin : zero;
    };
    set_tap(tap);

    auto issue = [&](int step) __attribute__((always_inline)) {
        const int stage = step % NS;
#pragma unroll
        // (the addresses go through named locals: with the sum written as the builtin's argument
        // the host pass drops the kernel's instantiation without a diagnostic)
        for (int j = 0; j < AJ; ++j) {
            const bf16* src = abase[j] + ci;
            __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(As + stage * BM * 32 +
                                                                                              (256 * j + wave * 64) * 8),
                                             16, 0, 0);
        }
        if (b_loader) {
            const bf16* src = bbase + ci;
            __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(Bs + stage * BN * 32 +
                                                                                              wave * 64 * 8),
                                             16, 0, 0);
        }
        ci += TK;
        if (ci >= a.Cin) {
            do {
                ci -= a.Cin;
                ++tap;
            } while (ci >= a.Cin);
            set_tap(tap);
        }
    };

    f4 acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const int wm = (wave / WGN) * (BM / WGM), wn = (wave % WGN) * (BN / WGN);

#pragma unroll
    for (int s = 0; s < NS - 1; ++s)
        if (s < nsteps) issue(s);
    for (int s = 0; s < nsteps; ++s) {
        // this wave's loads of step s have landed once at most the later steps' are outstanding
        const int later = min(nsteps - 1 - s, NS - 2);
        if (later >= NS - 2) {
            if (b_loader) asm volatile("s_waitcnt vmcnt(%0)" ::"n"((NS - 2) * (AJ + 1)) : "memory");
            else asm volatile("s_waitcnt vmcnt(%0)" ::"n"((NS - 2) * AJ) : "memory");
        } else {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        }
        // A plain hardware barrier: the LDS data of step s came from the direct loads just waited
        // for, and the loop writes LDS no other way, so the workgroup fence of __syncthreads (which
        // would also wait for the loads still in flight for later steps) is not needed; the empty
        // asm keeps the compiler from moving LDS accesses across it.
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        // every wave is past step s - 1: its stage takes the loads of step s + NS - 1
        if (s + NS - 1 < nsteps) issue(s + NS - 1);
        const bf16* A = As + (s % NS) * BM * 32;
        const bf16* B = Bs + (s % NS) * BN * 32;
        bf16x8 fb[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            fb[j] = *reinterpret_cast<const bf16x8*>(B + conv_slot(wn + 16 * j + lane % 16, lane / 16) * 8);
#pragma unroll
        for (int i = 0; i < MI; ++i) {
            const bf16x8 fa = *reinterpret_cast<const bf16x8*>(A + conv_slot(wm + 16 * i + lane % 16, lane / 16) * 8);
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[j], acc[i][j], 0, 0, 0);
        }
    }
    // result: lane holds column lane % 16, rows 4 (lane / 16) + r
    if (a.part) {
        float* out = a.part + size_t(blockIdx.z) * P * a.Cout;
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int col = n0 + wn + 16 * j + lane % 16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + wm + 16 * i + 4 * (lane / 16) + r;
                    if (row < P && col < a.Cout) out[size_t(row) * a.Cout + col] = acc[i][j][r];
                }
            }
        return;
    }
    if (a.y.p && !a.yf && a.Cout % 8 == 0 && a.y.cs % 8 == 0 && a.y.co % 8 == 0) {
        // bf16 output through LDS (free after the K loop): the tile is written back in rows of
        // 16-byte chunks instead of one 2-byte store per accumulator element
        constexpr int BNP = BN + 8;  // padded LDS row (a multiple of 16 bytes)
        static_assert(BM * BNP * 2 <= NS * (BM + BN) * 64, "the output tile fits the operand stages");
        bf16* Cs = reinterpret_cast<bf16*>(smem);
        __syncthreads();  // every wave is done with the operand stages
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int cl = wn + 16 * j + lane % 16;
                const float b = (a.bias && n0 + cl < a.Cout) ? a.bias[n0 + cl] : 0.f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float v = acc[i][j][r] + b;
                    if (a.relu) v = fmaxf(v, 0.f);
                    Cs[(wm + 16 * i + 4 * (lane / 16) + r) * BNP + cl] = bf16(v);
                }
            }
        __syncthreads();
        constexpr int G = BN / 8;  // 8-channel chunks per tile row
#pragma unroll
        for (int c = tid; c < BM * G; c += 256) {
            const int rl = c / G, g = c % G;
            const int row = m0 + rl, col = n0 + 8 * g;
            if (row < P && col < a.Cout)
                *reinterpret_cast<bf16x8*>(a.y.p + size_t(row) * a.y.cs + a.y.co + col) =
                    *reinterpret_cast<const bf16x8*>(Cs + rl * BNP + 8 * g);
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int col = n0 + wn + 16 * j + lane % 16;
            if (col >= a.Cout) continue;
            const float b = a.bias ? a.bias[col] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + 16 * i + 4 * (lane / 16) + r;
                if (row >= P) continue;
                float v = acc[i][j][r] + b;
                if (a.relu) v = fmaxf(v, 0.f);
                if (a.y.p) a.y.p[size_t(row) * a.y.cs + a.y.co + col] = bf16(v);
                if (a.yf) a.yf[size_t(row) * a.Cout + col] = v;
            }
        }
}

// LDS rows of the halo-tile kernel: a row (one pixel's or one output channel's 32-channel chunk,
// four 16-byte K groups) takes five 16-byte slots.  The 80-byte stride puts the 16-byte reads of any
// 16 consecutive rows (one MFMA operand, which starts at any pixel shift) in distinct banks, and a
// read's address is a per-lane base plus a constant.
constexpr int kTileRow = 5;

// Output of a halo tile (k_conv_tile).  Lane (wave row wr, wave channel group wc)
// holds, for fragment (i, g, j), output channel n0 + wc CW + 16 j + lane % 16 of the pixels
// 4 (lane / 16) + r, r < 4, of tile row wr RW + i, columns 16 g + ...: each lane computes one
// base address, and the offsets of its elements are uniform products (scalar arithmetic).  bf16
// outputs go through LDS (the operand stages, free once every wave is past its last multiply) and
// leave in 16-byte row chunks; fp32 outputs and split partials are stored from the registers.
template <int TH, int TW, int BN, int WR, int LDSB, int RW = TH / WR, int CG = TW / 16, int NJ = BN / (4 / WR) / 16>
__device__ __forceinline__ void tile_epilogue(const ConvArgs& a, const f4 (&acc)[RW][CG][NJ], bf16x8* lds,
                                              int n, int y0, int x0, int n0, int wr, int wc, int lane, int tid)
{
    constexpr int CW = 16 * NJ;
    const size_t W = size_t(a.W), Cout = size_t(a.Cout);
    const int cl0 = wc * CW + lane % 16;
    const size_t pix0 = (size_t(n) * a.H + y0 + wr * RW) * W + x0 + 4 * (lane / 16);
    // pixel of element (i, g, r) = pix0 + off(i, g, r)
    auto off = [&](int i, int g, int r) __attribute__((always_inline)) { return size_t(i) * W + 16 * g + r; };
    if (a.part) {
        float* out = a.part + (size_t(blockIdx.z) * a.N * a.H * W + pix0) * Cout + n0 + cl0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            if (n0 + cl0 + 16 * j >= a.Cout) continue;
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int g = 0; g < CG; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) out[off(i, g, r) * Cout + 16 * j] = acc[i][g][j][r];
        }
        return;
    }
    float bias[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int col = n0 + cl0 + 16 * j;
        bias[j] = (a.bias && col < a.Cout) ? a.bias[col] : 0.f;
    }
    auto act = [&](float v) __attribute__((always_inline)) { return a.relu ? fmaxf(v, 0.f) : v; };
    if (a.yf) {
        float* out = a.yf + pix0 * Cout + n0 + cl0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            if (n0 + cl0 + 16 * j >= a.Cout) continue;
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int g = 0; g < CG; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) out[off(i, g, r) * Cout + 16 * j] = act(acc[i][g][j][r] + bias[j]);
        }
    }
    if (!a.y.p) return;
    const size_t cs = size_t(a.y.cs);
    if (a.Cout % 8 || a.y.cs % 8 || a.y.co % 8) {
        bf16* out = a.y.p + pix0 * cs + a.y.co + n0 + cl0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            if (n0 + cl0 + 16 * j >= a.Cout) continue;
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int g = 0; g < CG; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) out[off(i, g, r) * cs + 16 * j] = bf16(act(acc[i][g][j][r] + bias[j]));
        }
        return;
    }
    constexpr int BNP = BN + 8;  // padded LDS row of the staged tile
    constexpr int G = BN / 8, PPI = 256 / G;  // 16-byte chunks per pixel, pixels per pass of the block
    static_assert(PPI % TW == 0 && (TH * TW) % PPI == 0, "whole tile rows per pass");
    static_assert(TH * TW * BNP * 2 <= LDSB, "the staged tile fits the operand stages");
    bf16* Cs = reinterpret_cast<bf16*>(lds);
    __syncthreads();  // every wave is done with the operand stages
    bf16* cw = Cs + (wr * RW * TW + 4 * (lane / 16)) * BNP + cl0;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int i = 0; i < RW; ++i)
#pragma unroll
            for (int g = 0; g < CG; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) cw[(i * TW + 16 * g + r) * BNP + 16 * j] = bf16(act(acc[i][g][j][r] + bias[j]));
    __syncthreads();
    if constexpr (BN == 32) {
        if (a.w1) {
            // the 1x1 convolution: one 16x16x32 MFMA per 16 staged pixels (the products and the
            // order of the pixel-row kernel with one K step); wave w takes a quarter of the pixels
            constexpr int PW = TH * TW / 4;
            const int o = lane % 16;
            bf16x8 wb;
#pragma unroll
            for (int e = 0; e < 8; ++e) wb[e] = bf16(0.f);
            if (o < a.c1) wb = *reinterpret_cast<const bf16x8*>(a.w1 + o * 32 + 8 * (lane / 16));
            const float b1 = (a.b1 && o < a.c1) ? a.b1[o] : 0.f;
            const int wave = tid / 64;
#pragma unroll
            for (int m = 0; m < PW / 16; ++m) {
                const int pb = wave * PW + 16 * m;
                const bf16x8 fa = *reinterpret_cast<const bf16x8*>(Cs + (pb + lane % 16) * BNP + 8 * (lane / 16));
                const f4 c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, wb, f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                if (o < a.c1) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int pl = pb + 4 * (lane / 16) + r;
                        a.y1[((size_t(n) * a.H + y0 + pl / TW) * W + x0 + pl % TW) * a.c1 + o] = c[r] + b1;
                    }
                }
            }
        }
    }
    const int p0 = tid / G, g8 = tid % G, col = n0 + 8 * g8;
    if (col >= a.Cout) return;
    const bf16* src = Cs + p0 * BNP + 8 * g8;
    bf16* dst = a.y.p + ((size_t(n) * a.H + y0 + p0 / TW) * W + x0 + p0 % TW) * cs + a.y.co + col;
#pragma unroll
    for (int k = 0; k < TH * TW / PPI; ++k)
        *reinterpret_cast<bf16x8*>(dst + size_t(k * (PPI / TW)) * W * cs) =
            *reinterpret_cast<const bf16x8*>(src + k * PPI * BNP);
    if (!a.pool.p) return;
    // 2x2 mean pooling of the staged tile (the same sums in the same order as k_pool_fwd); item
    // tid + 256 k is pooled pixel (tid + 256 k) / G, chunk g8 (G divides 256, so the chunk and the
    // column test above are this thread's for every k)
    constexpr int TWp = TW / 2, NP = TH * TW / 4;
    static_assert(TH % 2 == 0 && (NP * G) % 256 == 0, "whole pooled tile per pass count");
    const size_t Wp = W / 2, ps = size_t(a.pool.cs);
#pragma unroll
    for (int k = 0; k < NP * G / 256; ++k) {
        const int q = (tid + 256 * k) / G, py = q / TWp, px = q % TWp;
        const bf16* ps0 = Cs + (2 * py * TW + 2 * px) * BNP + 8 * g8;
        float acc8[8] = {};
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const bf16x8 v = *reinterpret_cast<const bf16x8*>(ps0 + (dy * TW + dx) * BNP);
#pragma unroll
                for (int e = 0; e < 8; ++e) acc8[e] += float(v[e]);
            }
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = bf16(0.25f * acc8[e]);
        *reinterpret_cast<bf16x8*>(a.pool.p + ((size_t(n) * (a.H / 2) + y0 / 2 + py) * Wp + x0 / 2 + px) * ps +
                                   a.pool.co + col) = o;
    }
}

// 3x3 convolution on spatial tiles (same result as k_conv_fwd<9, ...>, with a.kper in channels).
// A block computes TH x TW output pixels of one image (H and W multiples of the tile) and BN output
// channels.  K runs over 32-channel chunks of the input; per chunk, the block stages the input
// halo tile ((TH + 2) x (TW + 2) pixels, periodic or zero edges) and the weights of all nine taps
// in LDS, then every tap reads its operand as a shifted window of the halo tile.  The input is thus
// read once per chunk instead of once per tap, and each wave does 9 RW (TW / 16) (CW / 16) MFMAs
// per barrier: the K step of the pixel-row kernel above gives 4-8, too few to cover the load
// latency and the barrier.  Waves form a WR x (4 / WR) grid over tile rows x output channels; a
// wave reads each halo-row window once and applies it to up to three of its output rows.  NS
// stages: 2, the next chunk's direct loads are issued right after the barrier; 1, they are issued
// after the chunk's multiplies, behind a second barrier (half the LDS, so more blocks per CU overlap
// one block's loads with the others' multiplies).  ONE: the block's K is a single chunk (no reload
// code, whose live source addresses would cost registers).
// Thread t fills the 16-byte slots 256 j + t of each stage (the lane order of its wave's direct
// loads); a slot's row and K group fix the source address, which is set once and then advanced
// by the chunk offset (the fifth slot of a row, padding, loads zeros).
template <int TH, int TW, int BN, int WR, int NS, bool ONE>
__global__ void __launch_bounds__(256) k_conv_tile(const ConvArgs a)
{
    constexpr int WC = 4 / WR, RW = TH / WR, CW = BN / WC, CG = TW / 16, NJ = CW / 16;
    constexpr int HW = TW + 2, HP = (TH + 2) * HW;
    constexpr int JA = (kTileRow * HP + 255) / 256, JB = (kTileRow * 9 * BN + 255) / 256;
    constexpr int SA = JA * 256, SS = SA + JB * 256;  // 16-byte slots: input part, one stage
    static_assert(WR * WC == 4 && RW * WR == TH && CW * WC == BN && NJ * 16 == CW && CG * 16 == TW, "tile shape");
    static_assert(NS == 1 || NS == 2, "one or two stages");
    static_assert(!(ONE && NS == 2), "a single chunk needs one stage");
    static_assert(NS * SS * 16 <= 163840, "LDS");
    __shared__ __align__(16) bf16x8 lds[NS * SS];
    const int tid = threadIdx.x, lane = tid % 64;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const int tiles_x = a.W / TW, tiles_y = a.H / TH;
    const int tx = blockIdx.x % tiles_x, ty = (blockIdx.x / tiles_x) % tiles_y, n = blockIdx.x / (tiles_x * tiles_y);
    const int y0 = ty * TH, x0 = tx * TW, n0 = blockIdx.y * BN;
    const int c_begin = a.part ? blockIdx.z * a.kper : 0;
    const int c_end = a.part ? min(a.Cin, c_begin + a.kper) : a.Cin;
    const int nsteps = ONE ? 1 : (c_end - c_begin + TK - 1) / TK;
    const bf16* zero = g_zero;
    // slot 256 j + t: row (256 j + t) / 5, K group (256 j + t) % 5 (4: padding)
    const bf16* asrc[JA];
    const bf16* bsrc[JB];
    int aq8[JA], bq8[JB];
    // input sources of the halo slots: x, or (chunks below a.cup) the upsampled low-resolution
    // image, whose pixel (yy / 2, xx / 2) a full-resolution pixel repeats
    auto set_a = [&](bool from_up) __attribute__((always_inline)) {
        const unsigned img = unsigned(n) * unsigned(a.H) * unsigned(a.W);  // first pixel of image n
        const unsigned Wl = unsigned(a.W / 2), imgl = unsigned(n) * unsigned(a.H / 2) * Wl;
#pragma unroll
        for (int j = 0; j < JA; ++j) {
            const int sl = 256 * j + tid, r = sl / kTileRow, q = sl - r * kTileRow;
            const int hy = r / HW, hx = r - hy * HW;
            int yy = y0 - 1 + hy, xx = x0 - 1 + hx;
            if (a.periodic) {
                yy = yy < 0 ? yy + a.H : (yy >= a.H ? yy - a.H : yy);
                xx = xx < 0 ? xx + a.W : (xx >= a.W ? xx - a.W : xx);
            }
            const bool in = q < 4 && r < HP && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
            aq8[j] = q < 4 ? 8 * q : 0;
            const bf16* src;
            if (from_up) {
                const unsigned pl = imgl + __umul24(unsigned(yy >> 1), Wl) + unsigned(xx >> 1);
                src = in ? a.up.p + size_t(pl) * unsigned(a.up.cs) + a.up.co : zero;
            } else {
                const unsigned pix = img + __umul24(unsigned(yy), unsigned(a.W)) + unsigned(xx);
                src = in ? a.x.p + size_t(pix) * unsigned(a.x.cs) + a.x.co : zero;
            }
            asrc[j] = src + aq8[j];
        }
    };
    set_a(a.up.p && c_begin < a.cup);
#pragma unroll
    for (int j = 0; j < JB; ++j) {
        const int sl = 256 * j + tid, r = sl / kTileRow, q = sl - r * kTileRow;
        const int t = r / BN, co = n0 + r - t * BN;
        const bool in = q < 4 && t < 9 && co < a.Cout;
        bq8[j] = q < 4 ? 8 * q : 0;
        bsrc[j] = (in ? a.w + size_t(unsigned(t * a.Cout + co)) * unsigned(a.Cin) : zero) + bq8[j];
    }

    auto issue = [&](int step) __attribute__((always_inline)) {
        bf16x8* A = lds + (step % NS) * SS + 64 * wave;
        const int c = c_begin + step * TK;
        if (a.up.p && step > 0 && c == a.cup) set_a(false);  // the skip channels start here
        if (c + TK <= c_end) {
#pragma unroll
            for (int j = 0; j < JA; ++j) {
                const bf16* src = asrc[j] + c;
                __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(A + 256 * j), 16, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                const bf16* src = bsrc[j] + c;
                __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(A + SA + 256 * j), 16, 0, 0);
            }
        } else {  // a short last chunk: the groups past its end load zeros
#pragma unroll
            for (int j = 0; j < JA; ++j) {
                const bf16* src = c + aq8[j] < c_end ? asrc[j] + c : zero;
                __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(A + 256 * j), 16, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                const bf16* src = c + bq8[j] < c_end ? bsrc[j] + c : zero;
                __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(A + SA + 256 * j), 16, 0, 0);
            }
        }
    };

    const int wr = wave / WC, wc = wave % WC;
    // this lane's operand rows: halo row wr RW + h, column 16 g + dx + lane % 16 (group lane / 16);
    // weight row t BN + wc CW + 16 j + lane % 16
    const int a_lane = ((wr * RW) * HW + lane % 16) * kTileRow + lane / 16;
    const int b_lane = SA + (wc * CW + lane % 16) * kTileRow + lane / 16;
    f4 acc[RW][CG][NJ];
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
        for (int g = 0; g < CG; ++g)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[i][g][j] = f4{0.f, 0.f, 0.f, 0.f};

    issue(0);
    for (int s = 0; s < nsteps; ++s) {
        // this thread's loads of chunk s have landed (the next chunk's are issued below); the
        // barrier makes every thread's visible and frees the other stage (its chunk is done)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (NS == 2 && s + 1 < nsteps) issue(s + 1);
        const bf16x8* St = lds + (s % NS) * SS;
        const bf16x8* A = St + a_lane;
        const bf16x8* B = St + b_lane;
        bf16x8 fb[9][NJ];
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int j = 0; j < NJ; ++j) fb[t][j] = B[(t * BN + 16 * j) * kTileRow];
        // halo row h of this wave (tile row wr RW + h - 1) feeds output row i through tap row h - i
#pragma unroll
        for (int h = 0; h < RW + 2; ++h)
#pragma unroll
            for (int g = 0; g < CG; ++g)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const bf16x8 fa = A[(h * HW + 16 * g + dx) * kTileRow];
#pragma unroll
                    for (int i = 0; i < RW; ++i) {
                        if (h - i < 0 || h - i > 2) continue;
#pragma unroll
                        for (int j = 0; j < NJ; ++j)
                            acc[i][g][j] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[(h - i) * 3 + dx][j], acc[i][g][j], 0, 0, 0);
                    }
                }
        asm volatile("" ::: "memory");
        if (NS == 1 && !ONE && s + 1 < nsteps) {
            // one stage: every wave has read this chunk before the next one overwrites it
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            issue(s + 1);
        }
    }

    tile_epilogue<TH, TW, BN, WR, NS * SS * 16>(a, acc, lds, n, y0, x0, n0, wr, wc, lane, tid);
}

// Split-K epilogue: y = act(bias + sum over k of part[k]), partials summed in split order.
__global__ void __launch_bounds__(256) k_split_sum(const ConvArgs a, int splits)
{
    const size_t P = size_t(a.N) * a.H * a.W;
    const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= P * a.Cout) return;
    const int col = int(e % a.Cout);
    const size_t row = e / a.Cout;
    float v = a.bias ? a.bias[col] : 0.f;
    float s = 0.f;
    for (int k = 0; k < splits; ++k) s += a.part[size_t(k) * P * a.Cout + e];
    v += s;
    if (a.relu) v = fmaxf(v, 0.f);
    if (a.y.p) a.y.p[row * a.y.cs + a.y.co + col] = bf16(v);
    if (a.yf) a.yf[e] = v;
}

// The same for four consecutive channels per thread (Cout, the output slice and the fp32 output
// aligned to four elements): 16-byte partial loads, the same sums in the same order.
__global__ void __launch_bounds__(256) k_split_sum4(const ConvArgs a, int splits)
{
    const size_t P = size_t(a.N) * a.H * a.W, n = P * a.Cout;
    const size_t e = 4 * (size_t(blockIdx.x) * 256 + threadIdx.x);
    if (e >= n) return;
    const int col = int(e % a.Cout);
    const size_t row = e / a.Cout;
    f4 s = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < splits; ++k) s += *reinterpret_cast<const f4*>(a.part + size_t(k) * n + e);
    f4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = (a.bias ? a.bias[col + i] : 0.f) + s[i];
        if (a.relu) v[i] = fmaxf(v[i], 0.f);
    }
    if (a.y.p) {
        bf16x4 o;
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = bf16(v[i]);
        *reinterpret_cast<bf16x4*>(a.y.p + row * a.y.cs + a.y.co + col) = o;
    }
    if (a.yf) *reinterpret_cast<f4*>(a.yf + e) = v;
}

void split_sum(const ConvArgs& a, int splits, hipStream_t st)
{
    const size_t n = size_t(a.N) * a.H * a.W * a.Cout;
    const bool vec = a.Cout % 4 == 0 && a.y.cs % 4 == 0 && a.y.co % 4 == 0 &&
                     reinterpret_cast<uintptr_t>(a.y.p) % 8 == 0 && reinterpret_cast<uintptr_t>(a.yf) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(a.part) % 16 == 0;
    if (vec)
        hipLaunchKernelGGL(k_split_sum4, dim3(unsigned((n / 4 + 255) / 256)), dim3(256), 0, st, a, splits);
    else
        hipLaunchKernelGGL(k_split_sum, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, a, splits);
}

struct WgradArgs {
    CSlice x;        // layer input, Cin channels
    CSlice dz;       // output gradient, Cout channels
    float* partial;  // [nsplit][taps][Cout][Cin]
    int N, H, W, Cin, Cout, chunk;  // chunk per split: pixels (a multiple of 64), or halo tiles
    int periodic;
    // input channels [0, cup) are the nearest 2x upsampling of up (H/2 x W/2; p null: none;
    // halo-tile kernel only, cup a multiple of 64)
    CSlice up;
    int cup;
};

// partial[s][tap][co][ci] = sum over the pixels p of split s of dz[p][co] x[p + off(tap)][ci].
// GEMM with M = Cout, N = Cin, K = pixels, in steps of TKW = 64 pixels (two 32-deep MFMA steps per
// barrier); grid (Cout / 64, Cin / 64, taps * nsplit), four waves each with a 32 x 32 part.  Both
// operands are transposed to pixel-contiguous LDS rows (row = channel): thread t loads, per step,
// the 8-channel group t % 8 of the pixel pair 2 (t / 8) .. +1 for both operands (16-byte loads, eight
// consecutive lanes covering one pixel's 64 channels) and writes each channel's two pixels as one
// 32-bit word.  Pixel k of row r sits in column (k + 8 sw(r)) mod 64, sw(r) = (r ^ (r >> 3)) & 7:
// the eight lanes of a pixel pair (rows 8 g + e) and the sixteen rows an MFMA operand read spans
// then fall in different banks, while each 8-pixel group stays one aligned 16-byte read.  The next
// step's operands are loaded into registers while the current step is multiplied, LDS is
// double-buffered (one barrier per step), and the pixel coordinates advance incrementally.
constexpr int TKW = 64;

__device__ __forceinline__ int wg_col(int r, int k) { return (k + 8 * ((r ^ (r >> 3)) & 7)) & (TKW - 1); }

template <int TAPS>
__global__ void __launch_bounds__(256) k_conv_wgrad(const WgradArgs a)
{
    __shared__ __align__(16) bf16 As[2][TM * TKW];
    __shared__ __align__(16) bf16 Bs[2][TN * TKW];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int P = a.N * a.H * a.W;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const int tap = blockIdx.z % TAPS, split = blockIdx.z / TAPS;
    const int dy = (TAPS == 9 ? tap / 3 - 1 : 0), dx = (TAPS == 9 ? tap % 3 - 1 : 0);
    const int pbeg = split * a.chunk, pend = min(P, pbeg + a.chunk);
    const int pp = tid / 8, cg = tid % 8;  // pixel pair of the step, 8-channel group
    const bool a_ok = m0 + 8 * cg < a.Cout, b_ok = n0 + 8 * cg < a.Cin;
    // coordinates of this thread's first pixel of the current step, advanced by TKW per step
    int p = pbeg + 2 * pp, pn = 0, py = 0, px = 0;
    if (p < P) decompose(p, a.H, a.W, pn, py, px);
    bf16x8 ra[2], rb[2];
    auto load = [&]() __attribute__((always_inline)) {
        int n = pn, y = py, x = px;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            ra[h] = bf16x8{};
            rb[h] = bf16x8{};
            if (p + h < pend) {
                if (a_ok) ra[h] = *reinterpret_cast<const bf16x8*>(a.dz.p + size_t(p + h) * a.dz.cs + a.dz.co + m0 + 8 * cg);
                int yy = y + dy, xx = x + dx;
                if (a.periodic) {
                    yy = yy < 0 ? yy + a.H : (yy >= a.H ? yy - a.H : yy);
                    xx = xx < 0 ? xx + a.W : (xx >= a.W ? xx - a.W : xx);
                }
                if (b_ok && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
                    rb[h] = *reinterpret_cast<const bf16x8*>(a.x.p + size_t((n * a.H + yy) * a.W + xx) * a.x.cs + a.x.co +
                                                             n0 + 8 * cg);
            }
            if (++x == a.W) {  // the pair's second pixel
                x = 0;
                if (++y == a.H) {
                    y = 0;
                    ++n;
                }
            }
        }
        // advance to the next step: TKW pixels further
        p += TKW;
        px += TKW;
        while (px >= a.W) {
            px -= a.W;
            if (++py == a.H) {
                py = 0;
                ++pn;
            }
        }
    };
    auto stash = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int r = 8 * cg + e;
            const int c = wg_col(r, 2 * pp);
            const __attribute__((ext_vector_type(2))) __bf16 wa = {ra[0][e], ra[1][e]};
            const __attribute__((ext_vector_type(2))) __bf16 wb = {rb[0][e], rb[1][e]};
            *reinterpret_cast<__attribute__((ext_vector_type(2))) __bf16*>(&As[buf][r * TKW + c]) = wa;
            *reinterpret_cast<__attribute__((ext_vector_type(2))) __bf16*>(&Bs[buf][r * TKW + c]) = wb;
        }
    };
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const int wm = (wave / 2) * 32, wn = (wave % 2) * 32;
    load();
    stash(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = pbeg; k0 < pend; k0 += TKW) {
        const bool more = k0 + TKW < pend;
        if (more) load();
#pragma unroll
        for (int h = 0; h < TKW / 32; ++h) {
            const int k = 32 * h + 8 * (lane / 16);
            bf16x8 fb[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int r = wn + 16 * j + lane % 16;
                fb[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][r * TKW + wg_col(r, k)]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int r = wm + 16 * i + lane % 16;
                const bf16x8 fa = *reinterpret_cast<const bf16x8*>(&As[buf][r * TKW + wg_col(r, k)]);
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[j], acc[i][j], 0, 0, 0);
            }
        }
        if (more) stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    float* out = a.partial + (size_t(split) * TAPS + tap) * size_t(a.Cout) * a.Cin;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + wn + 16 * j + lane % 16;  // ci
            if (col >= a.Cin) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + 16 * i + 4 * (lane / 16) + r;  // co
                if (row < a.Cout) out[size_t(row) * a.Cin + col] = acc[i][j][r];
            }
        }
}

// Weight gradient of a 3x3 convolution on spatial tiles: partial[s][tap][co][ci] = sum over the
// pixels p of the tiles of split s of dz[p][co] x[p + off(tap)][ci].  A block owns 64 output
// channels (m0) x 64 input channels (n0) and all nine taps, and walks the 128-pixel tiles
// (128 / TW rows x TW columns) of its split.  Per tile it stages dz (128 pixel rows) and the input
// halo tile (periodic or zero edges) in LDS in their natural pixel-major layout with 16-byte direct
// loads, the next two tiles' loads in flight during the current tile's multiplies (three stages,
// 52 KB each: one block per CU).  The
// GEMM has M = co, N = ci, K = pixels; its operands need eight consecutive pixels per lane, which
// the LDS transpose read (ds_read_b64_tr_b16) gives from pixel rows: within 16 lanes, lane i
// receives element i % 4 of the 8-byte chunks addressed by lanes 4 e + i / 4 (e < 4), so lanes
// addressing pixel rows P0 + j / 4 at channels c0 + 4 (j % 4) hand lane i channel c0 + i of pixels
// P0 .. P0 + 3.  K element e of lane group q maps to tile pixel 32 s + 16 (e / 4) + 4 q + e % 4;
// a tap shifts the input rows read, not their alignment.  Rows are 160 bytes (64 channels, 32
// bytes of padding): the 8 or 16 consecutive rows of one read then fall in distinct banks at any
// shift.  Wave w multiplies input-channel group w (16 channels) for every tap and each of the NG
// output groups (NG = 2 when the layer has at most 32 output channels): nine operand reads of x
// and NG of dz feed 9 NG MFMAs per 32 pixels.
constexpr int kWgRow = 10;  // 16-byte slots per LDS row

template <int TW, int NG>
__global__ void __launch_bounds__(256) k_wgrad_tile(const WgradArgs a)
{
    constexpr int TH = 128 / TW, HW = TW + 2, HP = (TH + 2) * HW, PT = TH * TW;
    constexpr int JD = (kWgRow * PT + 255) / 256, JX = (kWgRow * HP + 255) / 256;
    constexpr int SD = JD * 256, SS = SD + JX * 256;  // 16-byte slots: dz part, one stage
    constexpr int NS = 3;
    static_assert(PT == 128 && TW % 16 == 0, "128-pixel tiles of whole 16-pixel row segments");
    static_assert(NS * SS * 16 <= 163840, "LDS");
    __shared__ __align__(16) bf16x8 lds[NS * SS];
    const int tid = threadIdx.x, lane = tid % 64;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    const int tiles_x = a.W / TW, tiles_y = a.H / TH, ntiles = a.N * tiles_y * tiles_x;
    const int t_begin = blockIdx.z * a.chunk, t_end = min(ntiles, t_begin + a.chunk);
    const bf16* zero = g_zero;
    // slot 256 j + t: row (256 j + t) / 10 and 8-channel group (256 j + t) % 10 (8, 9: padding).
    // The tile-independent part of each slot's source, set once: dz slots keep their element offset
    // from the tile's first pixel, x slots their halo coordinates (hy << 16 | hx) and channel
    // offset; -1 marks padding, rows past the tile and channels past the tensor (zeros).
    int doff[JD], xhw[JX], xoff[JX];
    // this block's input channels come from x or, below a.cup, from the upsampled low-resolution
    // image (pixel (yy / 2, xx / 2))
    const bool from_up = a.up.p && n0 < a.cup;
    const bf16* xsrc = from_up ? a.up.p : a.x.p;
    const unsigned xcs = unsigned(from_up ? a.up.cs : a.x.cs);
#pragma unroll
    for (int j = 0; j < JD; ++j) {
        const int sl = 256 * j + tid, r = sl / kWgRow, q = sl - r * kWgRow;
        const bool in = q < 8 && r < PT && m0 + 8 * q < a.Cout;
        doff[j] = in ? ((r / TW) * a.W + r % TW) * a.dz.cs + a.dz.co + m0 + 8 * q : -1;
    }
#pragma unroll
    for (int j = 0; j < JX; ++j) {
        const int sl = 256 * j + tid, r = sl / kWgRow, q = sl - r * kWgRow;
        const bool in = q < 8 && r < HP && n0 + 8 * q < a.Cin;
        xhw[j] = in ? ((r / HW) << 16) | (r % HW) : -1;
        xoff[j] = (from_up ? a.up.co : a.x.co) + n0 + 8 * q;
    }
    auto issue = [&](int tl, int stage) __attribute__((always_inline)) {
        const int tx = tl % tiles_x, ty = (tl / tiles_x) % tiles_y, n = tl / (tiles_x * tiles_y);
        const int y0 = ty * TH, x0 = tx * TW;
        const int img = n * a.H * a.W;
        const bf16* dzb = a.dz.p + size_t(img + y0 * a.W + x0) * a.dz.cs;  // the tile's first pixel
        bf16x8* D = lds + stage * SS + 64 * wave;
#pragma unroll
        for (int j = 0; j < JD; ++j) {
            const bf16* src = doff[j] >= 0 ? dzb + doff[j] : zero;
            __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(D + 256 * j), 16, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < JX; ++j) {
            int yy = y0 - 1 + (xhw[j] >> 16), xx = x0 - 1 + (xhw[j] & 0xffff);
            if (a.periodic) {
                yy = yy < 0 ? yy + a.H : (yy >= a.H ? yy - a.H : yy);
                xx = xx < 0 ? xx + a.W : (xx >= a.W ? xx - a.W : xx);
            }
            const bool in = xhw[j] >= 0 && unsigned(yy) < unsigned(a.H) && unsigned(xx) < unsigned(a.W);
            const unsigned pix = from_up ? unsigned(img / 4) + __umul24(unsigned(yy >> 1), unsigned(a.W / 2)) + unsigned(xx >> 1)
                                         : unsigned(img) + __umul24(unsigned(yy), unsigned(a.W)) + unsigned(xx);
            const bf16* src = in ? xsrc + size_t(pix) * xcs + xoff[j] : zero;
            __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(D + SD + 256 * j), 16, 0, 0);
        }
    };

    typedef __attribute__((address_space(3))) __bf16 lbf16;
    typedef __attribute__((address_space(3))) bf16x4 lbf16x4;
    auto tr = [&](const lbf16* p) __attribute__((always_inline)) {
        return __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lbf16x4*)p);
    };
    // lane (group q, index j): pixel row 4 q + j / 4 of each 16-pixel half step, channels 4 (j % 4)
    const int q = lane / 16, jr = (lane % 16) / 4, jc = 4 * (lane % 4);
    // (a wave whose input-channel group lies past the tensor multiplies zeros on its own SIMD and
    // stores nothing)
    f4 acc[9][NG];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[t][g] = f4{0.f, 0.f, 0.f, 0.f};

    if (t_begin < t_end) issue(t_begin, 0);
    if (t_begin + 1 < t_end) issue(t_begin + 1, 1);
    for (int tl = t_begin, k = 0; tl < t_end; ++tl, ++k) {
        // this thread's loads of tile k have landed once at most those of tile k + 1 are
        // outstanding (loads complete in order; no stores in the loop)
        if (tl + 1 < t_end) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(JD + JX) : "memory");
        else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        // every wave is past tile k - 1: its stage takes tile k + 2
        if (tl + 2 < t_end) issue(tl + 2, (k + 2) % NS);
        const lbf16* St = (const lbf16*)(lds + (k % NS) * SS);
        {
#pragma unroll
            for (int s = 0; s < PT / 32; ++s) {
                // every operand read of the K step first (22 or 26 transpose reads), so that their
                // latency is paid once rather than before each tap's MFMAs
                bf16x4 alo[NG], ahi[NG], blo[9], bhi[9];
                const int p0 = 32 * s + 4 * q + jr, p1 = p0 + 16;  // tile pixels of the two halves
                const int x0r = (p0 / TW + 1) * HW + p0 % TW + 1, x1r = (p1 / TW + 1) * HW + p1 % TW + 1;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    alo[g] = tr(St + p0 * (8 * kWgRow) + 16 * g + jc);
                    ahi[g] = tr(St + p1 * (8 * kWgRow) + 16 * g + jc);
                }
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const lbf16* X = St + SD * 8 + 16 * wave + jc + ((t / 3 - 1) * HW + (t % 3 - 1)) * (8 * kWgRow);
                    blo[t] = tr(X + x0r * (8 * kWgRow));
                    bhi[t] = tr(X + x1r * (8 * kWgRow));
                }
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const bf16x8 fb = {blo[t][0], blo[t][1], blo[t][2], blo[t][3], bhi[t][0], bhi[t][1], bhi[t][2], bhi[t][3]};
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        const bf16x8 fa = {alo[g][0], alo[g][1], alo[g][2], alo[g][3], ahi[g][0], ahi[g][1], ahi[g][2], ahi[g][3]};
                        acc[t][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[t][g], 0, 0, 0);
                    }
                }
            }
        }
        asm volatile("" ::: "memory");
    }
    // C: lane holds input channel n0 + 16 wave + lane % 16 of output channels m0 + 16 g + 4 q + r
    const int ci = n0 + 16 * wave + lane % 16;
    if (ci >= a.Cin) return;
    float* out = a.partial + size_t(blockIdx.z) * 9 * size_t(a.Cout) * a.Cin + ci;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = m0 + 16 * g + 4 * q + r;
                if (co < a.Cout) out[(size_t(t) * a.Cout + co) * a.Cin] = acc[t][g][r];
            }
}

// grad[e] = sum over k < nsplit of partial[k][e]: L lanes per element (256 / L elements per block)
// summing interleaved k, then a butterfly over the L lanes (every lane forms the same sums in the
// same order, so the result does not depend on scheduling).  L = 8 keeps each load coalesced over
// eight consecutive elements; L = 64 (a wave per element) serves short outputs summed over many
// partials.  One thread per element walking all k was bound by the latency of its dependent loads.
template <int L>
__global__ void __launch_bounds__(256) k_sum_splits(const float* partial, int nsplit, size_t n, float* grad)
{
    const int l = threadIdx.x % L;
    const size_t e = size_t(blockIdx.x) * (256 / L) + threadIdx.x / L;
    float s = 0.f;
    if (e < n) {
        // four partial sums (k = l + L (4 i + u)) keep four loads in flight, then combined in order
        float u4[4] = {0.f, 0.f, 0.f, 0.f};
        int k = l;
        for (; k + 3 * L < nsplit; k += 4 * L)
#pragma unroll
            for (int u = 0; u < 4; ++u) u4[u] += partial[size_t(k + L * u) * n + e];
        if (k < nsplit) u4[0] += partial[size_t(k) * n + e];
        if (k + L < nsplit) u4[1] += partial[size_t(k + L) * n + e];
        if (k + 2 * L < nsplit) u4[2] += partial[size_t(k + 2 * L) * n + e];
        s = (u4[0] + u4[1]) + (u4[2] + u4[3]);
    }
#pragma unroll
    for (int m = 1; m < L; m *= 2) s += __shfl_xor(s, m);
    if (e < n && l == 0) grad[e] = s;
}

void sum_splits(const float* partial, int nsplit, size_t n, float* grad, hipStream_t st)
{
    if (n <= 4096 && nsplit >= 256)
        hipLaunchKernelGGL(k_sum_splits<64>, dim3(unsigned((n + 3) / 4)), dim3(256), 0, st, partial, nsplit, n, grad);
    else
        hipLaunchKernelGGL(k_sum_splits<8>, dim3(unsigned((n + 31) / 32)), dim3(256), 0, st, partial, nsplit, n, grad);
}

// Bias gradient partials: part[b][co] = sum of dz[p][co] over the pixels p of chunk b (chunk pixels
// each).  Eight channels per thread; the block's threads split the chunk into L = 256 / (Cout / 8)
// interleaved pixel lanes (one lane per thread when Cout > 2048), summed in a fixed order.
__global__ void __launch_bounds__(256) k_bias_partial(CSlice dz, int P, int Cout, int chunk, float* part)
{
    __shared__ float sh[256 * 8];
    const int G = Cout / 8;
    const int L = G >= 256 ? 1 : 256 / G;
    const int p0 = blockIdx.x * chunk, p1 = min(P, p0 + chunk);
    for (int g0 = 0; g0 < G; g0 += 256) {
        const int t = threadIdx.x, g = g0 + t % min(G, 256), lane = t / min(G, 256);
        float acc[8] = {};
        if (lane < L && g < G)
            for (int p = p0 + lane; p < p1; p += L) {
                const bf16x8 v = *reinterpret_cast<const bf16x8*>(dz.p + size_t(p) * dz.cs + dz.co + 8 * g);
#pragma unroll
                for (int k = 0; k < 8; ++k) acc[k] += float(v[k]);
            }
#pragma unroll
        for (int k = 0; k < 8; ++k) sh[t * 8 + k] = acc[k];
        __syncthreads();
        const int gs = min(G - g0, 256);
        for (int c = threadIdx.x; c < gs * 8; c += 256) {
            // channel c of this pass: group c / 8, lane sums in order
            float s = 0.f;
            for (int l = 0; l < L; ++l) s += sh[(l * min(G, 256) + c / 8) * 8 + c % 8];
            part[size_t(blockIdx.x) * Cout + 8 * g0 + c] = s;
        }
        __syncthreads();
    }
}

// Kernel for the input gradient: wt[tap][ci][co] = w[taps - 1 - tap][co][ci] (mirrored taps,
// channel roles exchanged), so the input gradient is a forward convolution of dz with wt.
template <typename T>
__global__ void __launch_bounds__(256) k_flip(const T* w, bf16* wt, int taps, int Cout, int Cin)
{
    const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= size_t(taps) * Cout * Cin) return;
    const int co = int(e % Cout);
    const size_t q = e / Cout;
    const int ci = int(q % Cin), tap = int(q / Cin);
    wt[e] = bf16(float(w[(size_t(taps - 1 - tap) * Cout + co) * Cin + ci]));
}

// The flips of every convolution of a network in one launch: element e of the concatenation of
// their wt arrays (convolution k owns [start[k], start[k + 1])), each as k_flip.
constexpr int kMaxFlip = 32;
struct FlipTable {
    int n;
    size_t start[kMaxFlip + 1];
    const float* w[kMaxFlip];
    bf16* wt[kMaxFlip];
    int taps[kMaxFlip], cout[kMaxFlip], cin[kMaxFlip];
};

__global__ void __launch_bounds__(256) k_flip_all(const FlipTable t)
{
    const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= t.start[t.n]) return;
    int k = 0;
    while (e >= t.start[k + 1]) ++k;
    const size_t l = e - t.start[k];
    const int Cout = t.cout[k], Cin = t.cin[k], taps = t.taps[k];
    const int co = int(l % Cout);
    const size_t q = l / Cout;
    const int ci = int(q % Cin), tap = int(q / Cin);
    t.wt[k][l] = bf16(t.w[k][(size_t(taps - 1 - tap) * Cout + co) * Cin + ci]);
}

// ------------------------------------------------------------------------ elementwise kernels

// The elementwise kernels below move eight channels (one 16-byte bf16x8) per thread: channel counts,
// slice offsets and strides are multiples of 8, so every group is one aligned vector access.
__device__ __forceinline__ bf16x8 ld8(const bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }
__device__ __forceinline__ void st8(bf16* p, bf16x8 v) { *reinterpret_cast<bf16x8*>(p) = v; }

// dz[p][c] = g[p][c] if y[p][c] > 0 else 0 (ReLU backward; dz contiguous with C channels)
// ReLU backward (as k_relu_bwd) with the bias gradient's partial sums: part[b][c] = sum of dz[p][c]
// over the pixels p of chunk b.  A block owns one chunk; thread t takes the 8-channel group
// t % G of the pixels t / G, t / G + L, ... (L = 256 / G pixel lanes, G = C / 8 <= 256), then the
// L lanes of each group are summed in lane order through LDS (the same sums on every run).
__global__ void __launch_bounds__(256) k_relu_bwd_bias(CSlice g, CSlice y, bf16* dz, int P, int C, int chunk,
                                                      float* part)
{
    __shared__ float red[256][9];
    const int G = C / 8, L = 256 / G;
    const int cg = threadIdx.x % G, lane = threadIdx.x / G, c = 8 * cg;
    float s[8] = {};
    const int p0 = blockIdx.x * chunk, p1 = min(P, p0 + chunk);
    if (lane < L)
        for (int p = p0 + lane; p < p1; p += L) {
            const bf16x8 yv = ld8(y.p + size_t(p) * y.cs + y.co + c), gv = ld8(g.p + size_t(p) * g.cs + g.co + c);
            bf16x8 o;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                o[k] = float(yv[k]) > 0.f ? gv[k] : bf16(0.f);
                s[k] += float(o[k]);
            }
            st8(dz + size_t(p) * C + c, o);
        }
#pragma unroll
    for (int k = 0; k < 8; ++k) red[threadIdx.x][k] = s[k];
    __syncthreads();
    for (int o = threadIdx.x; o < C; o += 256) {
        const int og = o / 8, ok = o % 8;
        float t = 0.f;
        for (int l = 0; l < L; ++l) t += red[l * G + og][ok];
        part[size_t(blockIdx.x) * C + o] = t;
    }
}

__global__ void __launch_bounds__(256) k_relu_bwd(CSlice g, CSlice y, bf16* dz, int P, int C)
{
    const int G = C / 8;
    const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= size_t(P) * G) return;
    const size_t p = e / G;
    const int c = int(e - p * G) * 8;
    const bf16x8 yv = ld8(y.p + p * y.cs + y.co + c), gv = ld8(g.p + p * g.cs + g.co + c);
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = float(yv[k]) > 0.f ? gv[k] : bf16(0.f);
    st8(dz + p * C + c, o);
}

// 2x2 average pooling: out (H/2 x W/2) from in (H x W)
__global__ void __launch_bounds__(256) k_pool_fwd(CSlice in, Slice out, int N, int H, int W, int C)
{
    const int Ho = H / 2, Wo = W / 2, G = C / 8;
    const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= size_t(N) * Ho * Wo * G) return;
    const int c = int(e % G) * 8;
    const size_t q = e / G;
    const int x = int(q % Wo), y = int((q / Wo) % Ho), n = int(q / (size_t(Wo) * Ho));
    float s[8] = {};
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            const bf16x8 v = ld8(in.p + size_t((n * H + 2 * y + dy) * W + 2 * x + dx) * in.cs + in.co + c);
#pragma unroll
            for (int k = 0; k < 8; ++k) s[k] += float(v[k]);
        }
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = bf16(0.25f * s[k]);
    st8(out.p + q * out.cs + out.co + c, o);
}

// gin[2y+dy][2x+dx][c] += gout[y][x][c] / 4   (gin at H x W)
__global__ void __launch_bounds__(256) k_pool_bwd_add(CSlice gout, Slice gin, int N, int H, int W, int C)
{
    const int G = C / 8;
    const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= size_t(N) * H * W * G) return;
    const int c = int(e % G) * 8;
    const size_t q = e / G;
    const int x = int(q % W), y = int((q / W) % H), n = int(q / (size_t(W) * H));
    const bf16x8 gv = ld8(gout.p + size_t((n * (H / 2) + y / 2) * (W / 2) + x / 2) * gout.cs + gout.co + c);
    bf16* t = gin.p + q * gin.cs + gin.co + c;
    const bf16x8 tv = ld8(t);
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = bf16(float(tv[k]) + 0.25f * float(gv[k]));
    st8(t, o);
}

// nearest 2x upsampling: out (2H x 2W) from in (H x W)
__global__ void __launch_bounds__(256) k_up_fwd(CSlice in, Slice out, int N, int H, int W, int C)
{
    const int H2 = 2 * H, W2 = 2 * W, G = C / 8;
    const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= size_t(N) * H2 * W2 * G) return;
    const int c = int(e % G) * 8;
    const size_t q = e / G;
    const int x = int(q % W2), y = int((q / W2) % H2), n = int(q / (size_t(W2) * H2));
    st8(out.p + q * out.cs + out.co + c, ld8(in.p + size_t((n * H + y / 2) * W + x / 2) * in.cs + in.co + c));
}

// gin[y][x][c] = sum of the four gout values it was copied to (gin at H x W)
__global__ void __launch_bounds__(256) k_up_bwd(CSlice gout, Slice gin, int N, int H, int W, int C)
{
    const int G = C / 8;
    const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= size_t(N) * H * W * G) return;
    const int c = int(e % G) * 8;
    const size_t q = e / G;
    const int x = int(q % W), y = int((q / W) % H), n = int(q / (size_t(W) * H));
    float s[8] = {};
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            const bf16x8 v = ld8(gout.p + size_t((n * 2 * H + 2 * y + dy) * 2 * W + 2 * x + dx) * gout.cs + gout.co + c);
#pragma unroll
            for (int k = 0; k < 8; ++k) s[k] += float(v[k]);
        }
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = bf16(s[k]);
    st8(gin.p + q * gin.cs + gin.co + c, o);
}

// Fluid pixel count of the mask, per 256-pixel block.
__global__ void __launch_bounds__(256) k_mask_count(const uint8_t* mask, int P, float* part)
{
    __shared__ float sh[256];
    const int p = blockIdx.x * 256 + threadIdx.x;
    sh[threadIdx.x] = (p < P && mask[p]) ? 1.f : 0.f;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out[0] = sum of part[0 .. n) in fp64, fixed order.
__global__ void __launch_bounds__(256) k_sum_partials(const float* part, int n, double* out)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// Masked squared error over the first `used` of C output channels: per-block sums of
// mask (y - t)^2 into part, and dz = 2 mask (y - t) / (count used) into the bf16 gradient.
__global__ void __launch_bounds__(256) k_mse(const float* y, const float* t, const uint8_t* mask, int P, int C,
                                             int used, const double* count, bf16* dz, float* part)
{
    __shared__ float sh[256];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const float inv = float(1.0 / (fmax(count[0], 1.0) * used));
    float s = 0.f;
    if (p < P) {
        const bool m = mask[p] != 0;
        for (int c = 0; c < C; ++c) {
            float g = 0.f;
            if (m && c < used) {
                const float d = y[size_t(p) * C + c] - t[size_t(p) * used + c];
                s += d * d;
                g = 2.f * d * inv;
            }
            dz[size_t(p) * C + c] = bf16(g);
        }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Adam on fp32 master parameters, then the bf16 copy used by the forward pass.
__global__ void __launch_bounds__(256) k_adam(float* w, float* m, float* v, const float* g, bf16* wb, size_t n,
                                              float lr, float b1, float b2, float eps, float c1, float c2)
{
    const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= n) return;
    const float gr = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gr;
    const float vv = b2 * v[e] + (1.f - b2) * gr * gr;
    m[e] = mm;
    v[e] = vv;
    const float ww = w[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    w[e] = ww;
    wb[e] = bf16(ww);
}

__global__ void __launch_bounds__(256) k_to_bf16(const float* w, bf16* wb, size_t n)
{
    const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (e < n) wb[e] = bf16(w[e]);
}

// -------------------------------------------------------------- features and initial fields

__global__ void __launch_bounds__(256) k_feat_sites(const uint8_t* solid, int n, float f_kn, float f_ax, float f_ay,
                                                    bf16* x, int C)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const float fl = solid[s] ? 0.f : 1.f;
    bf16* o = x + size_t(s) * C;
    for (int c = 0; c < C; ++c) {
        float v = 0.f;
        if (c <= 8) v = fl;
        else if (c == 9) v = f_kn;
        else if (c == 10) v = f_ax;
        else if (c == 11) v = f_ay;
        o[c] = bf16(v);
    }
}

__global__ void __launch_bounds__(256) k_feat_links(const lbm_link* links, int64_t nl, const uint8_t* solid, int nx,
                                                    int ny, bf16* x, int C)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= nl) return;
    const lbm_link l = links[i];
    if (l.x < 0 || l.x >= nx || l.y < 0 || l.y >= ny || l.dir < 1 || l.dir > 8) return;
    const size_t s = size_t(l.y) * nx + l.x;
    if (solid[s]) return;
    x[s * C + l.dir] = bf16(float(l.q));
}

// Unpacks one predicted image into three fp64 planes (u_x, u_y, density deviation) over fluid
// sites, 0 on solid sites.
__global__ void __launch_bounds__(256) k_unpack(const float* pred, int stride, const uint8_t* solid, int n, double* t)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const bool fl = !solid[s];
    for (int c = 0; c < 3; ++c) t[size_t(c) * n + s] = fl ? double(pred[size_t(s) * stride + c]) : 0.0;
}

// One smoothing pass: at a fluid site, the mean of the three planes over the fluid sites of its
// 3 x 3 neighbourhood (rows and columns wrap around when periodic, else the image edge bounds
// the neighbourhood); 0 on solid sites.
__global__ void __launch_bounds__(256) k_smooth(const double* in, double* out, const uint8_t* solid, int nx, int ny,
                                                int periodic)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int n = nx * ny;
    if (s >= n) return;
    const int y = s / nx, x = s - y * nx;
    double acc[3] = {0.0, 0.0, 0.0};
    int cnt = 0;
    if (!solid[s]) {
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int yy = y + dy, xx = x + dx;
                if (periodic) {
                    yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
                    xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
                }
                if (yy < 0 || yy >= ny || xx < 0 || xx >= nx) continue;
                const int q = yy * nx + xx;
                if (solid[q]) continue;
                ++cnt;
                for (int c = 0; c < 3; ++c) acc[c] += in[size_t(c) * n + q];
            }
    }
    for (int c = 0; c < 3; ++c) out[size_t(c) * n + s] = cnt ? acc[c] / cnt : 0.0;
}

// One block: mean of the density deviation over fluid sites (fp64, fixed order), then the
// fields.  bad[0] = fluid sites with a non-finite value.
__global__ void __launch_bounds__(1024) k_fields(const double* t, const uint8_t* solid, int n, double us, double rs,
                                                 double rho0, double* rho, double* ux, double* uy, long long* bad)
{
    __shared__ double s_sum[1024];
    __shared__ int s_cnt[1024], s_bad[1024];
    const int tid = threadIdx.x;
    double sum = 0.0;
    int cnt = 0, nb = 0;
    for (int s = tid; s < n; s += 1024) {
        if (solid[s]) continue;
        const double a = t[s], b = t[size_t(n) + s], c = t[2 * size_t(n) + s];
        if (!isfinite(a) || !isfinite(b) || !isfinite(c)) {
            ++nb;
        } else {
            sum += c;
            ++cnt;
        }
    }
    s_sum[tid] = sum;
    s_cnt[tid] = cnt;
    s_bad[tid] = nb;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) {
            s_sum[tid] += s_sum[tid + w];
            s_cnt[tid] += s_cnt[tid + w];
            s_bad[tid] += s_bad[tid + w];
        }
        __syncthreads();
    }
    const double mean = s_cnt[0] ? s_sum[0] / s_cnt[0] : 0.0;
    for (int s = tid; s < n; s += 1024) {
        if (solid[s]) {
            rho[s] = rho0;
            ux[s] = 0.0;
            uy[s] = 0.0;
        } else {
            rho[s] = rho0 + rs * (t[2 * size_t(n) + s] - mean);
            ux[s] = us * t[s];
            uy[s] = us * t[size_t(n) + s];
        }
    }
    if (tid == 0) bad[0] = s_bad[0];
}

inline unsigned blocks(size_t n) { return unsigned((n + 255) / 256); }

// ------------------------------------------------------------------------------- launchers

// pipeline stages of the pixel-row convolution kernel (3 measured faster than 2 or 4)
constexpr int kConvStages = 3;

// Splits of the K range for a pixel-row convolution whose 64 x 64 grid has too few blocks to fill
// the chip: enough splits for about 1024 blocks, at most 8, each at least 16 K steps long (1 = no
// split).
int row_splits(long P, int Cin, int Cout, int taps)
{
    const long tiles = ((P + 63) / 64) * ((Cout + 63) / 64);
    if (Cout < 64 || tiles >= 1024) return 1;
    const int K = taps * Cin;
    int s = int(std::min<long>(8, 1024 / std::max<long>(tiles, 1)));
    while (s > 1 && K / s < 16 * TK) --s;
    return std::max(1, s);
}

// Kernel and K split of one forward convolution.  3x3 convolutions whose image is a whole number
// of tiles take the halo-tile kernel: 8 x 32 pixels x 64 channels when the output channels are a
// multiple of 64 and that still gives a block per compute unit (256), else 8 x 16 x 64, else
// 8 x 32 x 32.  K is split (over the workspace) when the grid has fewer than 256 blocks, at most 8
// ways and, with four or more chunks, at least two 32-channel chunks per split.  Measured at batch 8
// on 256^2: small tiles that put several blocks on a CU beat larger ones (8 x 32 x 32 with one
// reloaded LDS stage, three blocks per CU: 48 us for 96 -> 32 channels against 69 us for
// 16 x 32 x 32 tiles with two stages, one block per CU; 2-6% on the single-chunk 32-channel
// layers), while 8 x 16 x 64 tiles in place of 8 x 32 x 64 ones at 64^2 gained nothing.
struct FwdPlan {
    int kind;    // 0: pixel-row kernel; halo tiles 1: 8 x 32 x 64; 2: 8 x 16 x 64; 3: 8 x 32 x 32
    int splits;  // K splits, 1: none
    int kper;    // K per split: input channels (tiles) or (tap, channel) positions (pixel rows)
};

FwdPlan fwd_plan(int N, int H, int W, int Cin, int Cout, int taps)
{
    FwdPlan f{0, 1, 0};
    const long P = long(N) * H * W;
    if (taps == 9 && Cin + 32 <= kZeroElems && H < (1 << 24) && W < (1 << 24)) {
        auto nb = [&](int th, int tw, int bn) { return long(N) * (H / th) * (W / tw) * ((Cout + bn - 1) / bn); };
        long blocks = 0;
        if (Cout % 64 == 0 && H % 8 == 0 && W % 32 == 0 && nb(8, 32, 64) >= 256) {
            f.kind = 1;
            blocks = nb(8, 32, 64);
        } else if (Cout % 64 == 0 && H % 8 == 0 && W % 16 == 0) {
            f.kind = 2;
            blocks = nb(8, 16, 64);
        } else if (H % 8 == 0 && W % 32 == 0) {
            f.kind = 3;
            blocks = nb(8, 32, 32);
        }
        if (f.kind) {
            const int chunks = (Cin + TK - 1) / TK;
            int s = blocks >= 256 ? 1 : int(std::min<long>({8, (256 + blocks - 1) / blocks, long(chunks)}));
            if (chunks >= 4) s = std::min(s, chunks / 2);
            s = std::max(s, 1);
            f.kper = (chunks + s - 1) / s * TK;
            f.splits = (Cin + f.kper - 1) / f.kper;
            return f;
        }
    }
    f.splits = row_splits(P, Cin, Cout, taps);
    const int K = taps * Cin;
    f.kper = ((K + f.splits - 1) / f.splits + TK - 1) / TK * TK;
    f.splits = (K + f.kper - 1) / f.kper;
    return f;
}

size_t fwd_split_elems(int N, int H, int W, int Cin, int Cout, int taps)
{
    const FwdPlan f = fwd_plan(N, H, W, Cin, Cout, taps);
    return f.splits > 1 ? size_t(f.splits) * size_t(N) * H * W * size_t(Cout) : 0;
}

template <int TH, int TW, int BN, int WR>
void launch_tile(const ConvArgs& a, int nsplit, int chunks_per_block, hipStream_t st)
{
    const dim3 grid(unsigned(a.N * (a.H / TH) * (a.W / TW)), unsigned((a.Cout + BN - 1) / BN), unsigned(nsplit));
    // several chunks: one reloaded stage where the grid puts two or more blocks on each CU (half
    // the LDS lets them share it: 53-78 KB per block), else two stages, so that a lone block still
    // overlaps its next chunk's loads with its multiplies
    const long nblocks = long(grid.x) * grid.y * grid.z;
    if (chunks_per_block == 1)
        hipLaunchKernelGGL((k_conv_tile<TH, TW, BN, WR, 1, true>), grid, dim3(256), 0, st, a);
    else if (nblocks >= 512)
        hipLaunchKernelGGL((k_conv_tile<TH, TW, BN, WR, 1, false>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_conv_tile<TH, TW, BN, WR, 2, false>), grid, dim3(256), 0, st, a);
}

// pool.p non-null: also the 2x2 mean of the bf16 output y (H and W even) into pool, fused into the
// halo-tile kernel's output stage where that kernel runs unsplit, else a separate pass.
// Input channels [0, cup) given as the nearest 2x upsampling of src (an H/2 x W/2 image; p null:
// none).  cat is where the input tensor keeps those channels: the convolutions read them from src
// where their halo-tile kernels run, and the upsampled values are written to cat first otherwise.
struct UpSrc {
    CSlice src;
    int cup;
    Slice cat;
};

// writes the upsampled channels into cat when a kernel needs them there
hipError_t materialize(const UpSrc& u, int N, int H, int W, hipStream_t st)
{
    hipLaunchKernelGGL(k_up_fwd, dim3(blocks(size_t(N) * H * W * u.cup / 8)), dim3(256), 0, st, u.src, u.cat, N, H / 2,
                       W / 2, u.cup);
    return hipGetLastError();
}

// A 1x1 convolution that follows a forward convolution (w null: none): w [c][Cout] bf16, b [c] or
// null, y fp32 [pixels][c].
struct Out1 {
    const bf16* w;
    const float* b;
    float* y;
    int c;
};

hipError_t conv_forward(CSlice x, const bf16* w, const float* bias, Slice y, float* yf, int N, int H, int W, int Cin,
                        int Cout, int taps, bool relu, bool periodic, hipStream_t st, float* ws, size_t ws_elems,
                        Slice pool = Slice{nullptr, 0, 0}, Out1 o1 = Out1{nullptr, nullptr, nullptr, 0},
                        UpSrc up = UpSrc{CSlice{nullptr, 0, 0}, 0, Slice{nullptr, 0, 0}});

// pool.p non-null: also the 2x2 mean of the bf16 output y (H and W even) into pool, fused into the
// halo-tile kernel's output stage where that kernel runs unsplit, else a separate pass.  o1.w
// non-null: also the 1x1 convolution o1 of y (no activation), fused the same way for 32-channel
// outputs, else a separate convolution.
hipError_t conv_forward(CSlice x, const bf16* w, const float* bias, Slice y, float* yf, int N, int H, int W, int Cin,
                        int Cout, int taps, bool relu, bool periodic, hipStream_t st, float* ws, size_t ws_elems,
                        Slice pool, Out1 o1, UpSrc up)
{
    if (Cin + 8 > kZeroElems || Cin % 8 || Cout < 1) return hipErrorInvalidValue;
    if (pool.p && (!y.p || H % 2 || W % 2 || Cout % 8 || pool.cs % 8 || pool.co % 8)) return hipErrorInvalidValue;
    if (o1.w && (!y.p || !o1.y || o1.c < 1)) return hipErrorInvalidValue;
    ConvArgs a{x,       w,       bias, y,  yf, N, H, W, Cin, Cout, relu ? 1 : 0, periodic ? 1 : 0, nullptr, 0,
               Slice{nullptr, 0, 0}, nullptr, nullptr, nullptr, 0, CSlice{nullptr, 0, 0}, 0};
    if (up.src.p && (H % 2 || W % 2 || up.cup % 8 || up.cup > Cin || !up.cat.p)) return hipErrorInvalidValue;
    // pooling as a separate pass after the convolution (where the fused form does not apply)
    auto pool_pass = [&]() {
        if (!pool.p) return hipGetLastError();
        hipLaunchKernelGGL(k_pool_fwd, dim3(blocks(size_t(N) * (H / 2) * (W / 2) * Cout / 8)), dim3(256), 0, st,
                           CSlice{y.p, y.cs, y.co}, pool, N, H, W, Cout);
        return hipGetLastError();
    };
    // the 1x1 convolution as a separate pass
    auto out1_pass = [&]() {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess || !o1.w) return e;
        return conv_forward(CSlice{y.p, y.cs, y.co}, o1.w, o1.b, Slice{nullptr, 0, 0}, o1.y, N, H, W, Cout, o1.c, 1,
                            false, periodic, st, ws, ws_elems);
    };
    const long P = long(N) * H * W;
    const FwdPlan f = fwd_plan(N, H, W, Cin, Cout, taps);
    if (up.src.p) {
        if (f.kind && up.cup % TK == 0) {  // whole chunks from one source
            a.up = up.src;
            a.cup = up.cup;
        } else {
            const hipError_t e = materialize(up, N, H, W, st);
            if (e != hipSuccess) return e;
        }
    }
    // split K over the workspace when the plan asks for it and the workspace holds the partials
    const bool split = f.splits > 1 && ws && ws_elems >= fwd_split_elems(N, H, W, Cin, Cout, taps);
    if (split) {
        a.part = ws;
        a.kper = f.kper;
    }
    const int nsplit = split ? f.splits : 1;
    if (f.kind) {
        const int chunks = ((split ? f.kper : Cin) + TK - 1) / TK;
        // fused pooling needs the staged bf16 output stage of an unsplit tile launch
        const bool staged = !split && y.p && Cout % 8 == 0 && y.cs % 8 == 0 && y.co % 8 == 0;
        const bool fuse_pool = pool.p && staged;
        const bool fuse_1x1 = o1.w && staged && f.kind == 3 && Cout == 32 && o1.c <= 16;
        if (fuse_pool) a.pool = pool;
        if (fuse_1x1) {
            a.w1 = o1.w;
            a.b1 = o1.b;
            a.y1 = o1.y;
            a.c1 = o1.c;
        }
        if (f.kind == 1) launch_tile<8, 32, 64, 2>(a, nsplit, chunks, st);
        else if (f.kind == 2) launch_tile<8, 16, 64, 2>(a, nsplit, chunks, st);
        else launch_tile<8, 32, 32, 4>(a, nsplit, chunks, st);
        if (split) split_sum(a, nsplit, st);
        if (!fuse_pool) {
            const hipError_t e = pool_pass();
            if (e != hipSuccess) return e;
        }
        return fuse_1x1 ? hipGetLastError() : out1_pass();
    }
    if (split) {
        const dim3 grid(unsigned((P + 63) / 64), unsigned((Cout + 63) / 64), unsigned(nsplit));
        const size_t lds = size_t(kConvStages) * (64 + 64) * 64;
        if (taps == 9)
            hipLaunchKernelGGL((k_conv_fwd<9, 64, 64, kConvStages>), grid, dim3(256), lds, st, a);
        else
            hipLaunchKernelGGL((k_conv_fwd<1, 64, 64, kConvStages>), grid, dim3(256), lds, st, a);
        split_sum(a, nsplit, st);
        const hipError_t e = pool_pass();
        return e != hipSuccess ? e : out1_pass();
    }
    // the largest tile that still leaves about four blocks per compute unit (256 CUs)
    auto nblocks = [&](int bm, int bn) { return ((P + bm - 1) / bm) * ((Cout + bn - 1) / bn); };
    auto go = [&](auto kern, int bm, int bn) {
        const dim3 grid(unsigned((P + bm - 1) / bm), unsigned((Cout + bn - 1) / bn));
        hipLaunchKernelGGL(kern, grid, dim3(256), size_t(kConvStages) * (bm + bn) * 64, st, a);
    };
    const bool t9 = taps == 9;
    if (Cout >= 64 && nblocks(128, 64) >= 1024)
        t9 ? go(k_conv_fwd<9, 128, 64, kConvStages>, 128, 64) : go(k_conv_fwd<1, 128, 64, kConvStages>, 128, 64);
    else if (Cout >= 64)
        t9 ? go(k_conv_fwd<9, 64, 64, kConvStages>, 64, 64) : go(k_conv_fwd<1, 64, 64, kConvStages>, 64, 64);
    else if (nblocks(128, 32) >= 1024)
        t9 ? go(k_conv_fwd<9, 128, 32, kConvStages>, 128, 32) : go(k_conv_fwd<1, 128, 32, kConvStages>, 128, 32);
    else
        t9 ? go(k_conv_fwd<9, 64, 32, kConvStages>, 64, 32) : go(k_conv_fwd<1, 64, 32, kConvStages>, 64, 32);
    const hipError_t e = pool_pass();
    return e != hipSuccess ? e : out1_pass();
}

template <typename T>
hipError_t flip(const T* w, bf16* wt, int taps, int Cout, int Cin, hipStream_t st)
{
    hipLaunchKernelGGL(k_flip<T>, dim3(blocks(size_t(taps) * Cout * Cin)), dim3(256), 0, st, w, wt, taps, Cout, Cin);
    return hipGetLastError();
}

// Input gradient from the flipped kernel wt ([taps][Cin][Cout]): a forward convolution with the
// channel roles exchanged (the adjoint of a zero-padded or of a periodic convolution is the
// convolution with the mirrored kernel under the same edge rule).
hipError_t conv_dgrad(CSlice dz, const bf16* wt, Slice dx, int N, int H, int W, int Cin, int Cout, int taps,
                      bool periodic, hipStream_t st, float* ws, size_t ws_elems)
{
    return conv_forward(dz, wt, nullptr, dx, nullptr, N, H, W, Cout, Cin, taps, false, periodic, st, ws, ws_elems);
}

struct WgradPlan {
    int nsplit, chunk, nb, bchunk;
    int tile_w;  // 32 or 16: the halo-tile kernel with 128-pixel tiles that wide (chunk in tiles); 0:
                 // the pixel-row kernel (chunk in pixels)
    size_t per, elems;
};

// 3x3 weight gradients of images that are a whole number of 128-pixel tiles take the halo-tile
// kernel, split over the tiles for about 256 blocks (one per CU; at most 256 splits, at least two
// tiles each);
// the others the pixel-row kernel, split over the pixels for about 1024 (tap, tile, split) blocks,
// at least 256 pixels per split.  elems = workspace (split partials + bias partials).
WgradPlan wgrad_plan(int N, int H, int W, int Cin, int Cout, int taps)
{
    WgradPlan w{};
    const int P = N * H * W;
    w.nb = std::min(256, (P + 255) / 256);  // bias partials: at most 256 pixel chunks
    w.bchunk = (P + w.nb - 1) / w.nb;
    w.per = size_t(taps) * Cout * Cin;
    if (taps == 9 && H < (1 << 24) && W < (1 << 24)) {
        if (W % 32 == 0 && H % 4 == 0) w.tile_w = 32;
        else if (W % 16 == 0 && H % 8 == 0) w.tile_w = 16;
    }
    if (w.tile_w) {
        const int ntiles = N * (H / (128 / w.tile_w)) * (W / w.tile_w);
        const int blocks = ((Cout + 63) / 64) * ((Cin + 63) / 64);
        int s = std::min(256, std::max(1, (256 + blocks - 1) / blocks));
        s = std::min(s, std::max(1, ntiles / 2));
        w.chunk = (ntiles + s - 1) / s;
        w.nsplit = (ntiles + w.chunk - 1) / w.chunk;
        w.elems = size_t(w.nsplit) * w.per + size_t(w.nb) * Cout;
        return w;
    }
    const int tiles = taps * ((Cout + TM - 1) / TM) * ((Cin + TN - 1) / TN);
    const int target = std::max(1, std::min(1024 / tiles, P / 256));
    w.chunk = ((P + target - 1) / target + TKW - 1) / TKW * TKW;
    w.nsplit = std::max(1, (P + w.chunk - 1) / w.chunk);
    w.elems = size_t(target) * w.per + size_t(w.nb) * Cout;
    return w;
}

hipError_t conv_wgrad(CSlice x, CSlice dz, float* dw, float* db, float* work, int N, int H, int W, int Cin, int Cout,
                      int taps, bool periodic, hipStream_t st, UpSrc up = UpSrc{CSlice{nullptr, 0, 0}, 0, Slice{nullptr, 0, 0}})
{
    const int P = N * H * W;
    const WgradPlan pl = wgrad_plan(N, H, W, Cin, Cout, taps);
    WgradArgs a{x, dz, work, N, H, W, Cin, Cout, pl.chunk, periodic ? 1 : 0, CSlice{nullptr, 0, 0}, 0};
    if (up.src.p) {
        if (pl.tile_w && up.cup % 64 == 0 && H % 2 == 0 && W % 2 == 0) {  // whole 64-channel blocks from one source
            a.up = up.src;
            a.cup = up.cup;
        } else {
            const hipError_t e = materialize(up, N, H, W, st);
            if (e != hipSuccess) return e;
        }
    }
    if (pl.tile_w) {
        const dim3 grid((Cout + 63) / 64, (Cin + 63) / 64, pl.nsplit);
        const bool two = Cout <= 32;  // two output groups of 16 cover the layer
        if (pl.tile_w == 32 && two)
            hipLaunchKernelGGL((k_wgrad_tile<32, 2>), grid, dim3(256), 0, st, a);
        else if (pl.tile_w == 32)
            hipLaunchKernelGGL((k_wgrad_tile<32, 4>), grid, dim3(256), 0, st, a);
        else if (two)
            hipLaunchKernelGGL((k_wgrad_tile<16, 2>), grid, dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_wgrad_tile<16, 4>), grid, dim3(256), 0, st, a);
    } else {
        const dim3 grid((Cout + TM - 1) / TM, (Cin + TN - 1) / TN, taps * pl.nsplit);
        if (taps == 9)
            hipLaunchKernelGGL(k_conv_wgrad<9>, grid, dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL(k_conv_wgrad<1>, grid, dim3(256), 0, st, a);
    }
    sum_splits(work, pl.nsplit, pl.per, dw, st);
    if (db) {
        float* bpart = work + size_t(pl.nsplit) * pl.per;
        hipLaunchKernelGGL(k_bias_partial, dim3(pl.nb), dim3(256), 0, st, dz, P, Cout, pl.bchunk, bpart);
        sum_splits(bpart, pl.nb, size_t(Cout), db, st);
    }
    return hipGetLastError();
}

}  // namespace nn
}  // namespace lbm

// ================================================================================ network

namespace {

using lbm::nn::bf16;
using lbm::nn::CSlice;
using lbm::nn::Slice;

struct Conv {
    int taps = 0, cin = 0, cout = 0, level = 0;
    size_t w_off = 0, b_off = 0;  // offsets into the flat fp32 parameter vector
    bf16* w = nullptr;            // bf16 weights [taps][cout][cin]
    bf16* wt = nullptr;           // flipped weights [taps][cin][cout] for the input gradient
};

// One resolution level; activations and their gradients are bf16 NHWC for max_batch images.
struct Level {
    int H = 0, W = 0, C = 0, cin = 0;
    Conv c1, c2;  // encoder
    Conv d1, d2;  // decoder (levels above the bottleneck)
    bf16 *in = nullptr, *e1 = nullptr, *cat = nullptr, *e2 = nullptr, *d1o = nullptr, *d2o = nullptr;
    bf16 *g_in = nullptr, *g_e1 = nullptr, *g_cat = nullptr, *g_e2 = nullptr, *g_d1o = nullptr, *g_d2o = nullptr;
};

constexpr int kOutPad = 8;  // output channels of the last convolution (rows beyond out_channels stay 0)

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

struct lbm_nn {
    lbm_nn_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<Level> lv;
    Conv out;
    std::vector<Conv*> convs;
    size_t n_params = 0;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // fp32 master, gradient, Adam moments
    bf16* wb = nullptr;                                            // bf16 copy of every parameter
    bf16* wt_all = nullptr;                                        // flipped bf16 kernels
    bf16* dz = nullptr;       // pre-activation gradient of the convolution being differentiated
    float* work = nullptr;    // weight-gradient and split-K workspace
    size_t work_elems = 0;
    float* part = nullptr;    // loss / count partials
    float* yout = nullptr;    // last forward output, fp32 [P][kOutPad]
    bf16* g_out = nullptr;    // its gradient
    double* d_red = nullptr;  // [0] fluid count, [1] loss sum
    double* h_red = nullptr;  // pinned host copy
    int last_n = 0;
    int64_t adam_t = 0;
    std::vector<void*> allocs;
};

namespace {

int chan(const lbm_nn* n, int l) { return n->cfg.base_channels << l; }

void nn_release(lbm_nn* n)
{
    if (!n) return;
    {
        DeviceGuard g(n->device);
        ignore(hipStreamSynchronize(n->stream));
        for (void* p : n->allocs) ignore(hipFree(p));
        if (n->h_red) ignore(hipHostFree(n->h_red));
    }
    delete n;
}

template <typename T>
bool nn_alloc(lbm_nn* n, T** p, size_t elems)
{
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(elems, 1) * sizeof(T)) != hipSuccess) return false;
    n->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return true;
}

CSlice cs(const bf16* p, int c, int off = 0) { return CSlice{p, c, off}; }
Slice sl(bf16* p, int c, int off = 0) { return Slice{p, c, off}; }

const lbm::nn::UpSrc kNoUp{CSlice{nullptr, 0, 0}, 0, Slice{nullptr, 0, 0}};

hipError_t fwd(lbm_nn* n, const Conv& c, CSlice x, Slice y, float* yf, int N, int H, int W, bool relu,
               Slice pool = Slice{nullptr, 0, 0}, lbm::nn::Out1 o1 = lbm::nn::Out1{nullptr, nullptr, nullptr, 0},
               lbm::nn::UpSrc up = kNoUp)
{
    return lbm::nn::conv_forward(x, c.w, n->w + c.b_off, y, yf, N, H, W, c.cin, c.cout, c.taps, relu,
                                 n->cfg.periodic != 0, n->stream, n->work, n->work_elems, pool, o1, up);
}

hipError_t wgrad(lbm_nn* n, const Conv& c, CSlice x, CSlice dz, int N, int H, int W)
{
    return lbm::nn::conv_wgrad(x, dz, n->g + c.w_off, n->g + c.b_off, n->work, N, H, W, c.cin, c.cout, c.taps,
                               n->cfg.periodic != 0, n->stream);
}

// Backward of one convolution + ReLU.  g: gradient w.r.t. its output y (after ReLU), x: its
// input.  Writes its weight and bias gradients and, if gx.p, the gradient w.r.t. x.
// pixel chunks of the fused ReLU / bias-gradient pass: up to 1024 blocks, at least 128 pixels each
int relu_bias_chunks(int P) { return std::max(1, std::min(1024, (P + 127) / 128)); }

hipError_t conv_relu_bwd(lbm_nn* n, const Conv& c, CSlice x, CSlice y, CSlice g, Slice gx, int N, int H, int W,
                         lbm::nn::UpSrc up = kNoUp)
{
    const int P = N * H * W;
    const CSlice dz = cs(n->dz, c.cout);
    hipError_t e;
    if (c.cout <= 2048) {
        // ReLU backward with the bias gradient's chunk partials (in the workspace, summed before
        // the weight gradient reuses it), then the weight gradient alone
        const int nb = relu_bias_chunks(P), chunk = (P + nb - 1) / nb;
        hipLaunchKernelGGL(lbm::nn::k_relu_bwd_bias, dim3(nb), dim3(256), 0, n->stream, g, y, n->dz, P, c.cout, chunk,
                           n->work);
        lbm::nn::sum_splits(n->work, nb, size_t(c.cout), n->g + c.b_off, n->stream);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = lbm::nn::conv_wgrad(x, dz, n->g + c.w_off, nullptr, n->work, N, H, W, c.cin, c.cout, c.taps,
                                n->cfg.periodic != 0, n->stream, up);
    } else {
        hipLaunchKernelGGL(lbm::nn::k_relu_bwd, dim3(lbm::nn::blocks(size_t(P) * c.cout / 8)), dim3(256), 0, n->stream,
                           g, y, n->dz, P, c.cout);
        e = hipGetLastError();
        if (e == hipSuccess && up.src.p) e = lbm::nn::materialize(up, N, H, W, n->stream);
        if (e != hipSuccess) return e;
        e = wgrad(n, c, x, dz, N, H, W);
    }
    if (e != hipSuccess || !gx.p) return e;
    return lbm::nn::conv_dgrad(dz, c.wt, gx, N, H, W, c.cin, c.cout, c.taps, n->cfg.periodic != 0, n->stream,
                               n->work, n->work_elems);
}

hipError_t refresh_flipped(lbm_nn* n)
{
    if (n->convs.size() > size_t(lbm::nn::kMaxFlip)) {
        for (Conv* cv : n->convs) {
            hipError_t e = lbm::nn::flip(n->w + cv->w_off, cv->wt, cv->taps, cv->cout, cv->cin, n->stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    lbm::nn::FlipTable t{};
    t.n = int(n->convs.size());
    for (int k = 0; k < t.n; ++k) {
        const Conv* cv = n->convs[k];
        t.w[k] = n->w + cv->w_off;
        t.wt[k] = cv->wt;
        t.taps[k] = cv->taps;
        t.cout[k] = cv->cout;
        t.cin[k] = cv->cin;
        t.start[k + 1] = t.start[k] + size_t(cv->taps) * cv->cout * cv->cin;
    }
    hipLaunchKernelGGL(lbm::nn::k_flip_all, dim3(lbm::nn::blocks(t.start[t.n])), dim3(256), 0, n->stream, t);
    return hipGetLastError();
}

bool conv_sizes_ok(int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout, int32_t ksize)
{
    return n >= 1 && h >= 1 && wd >= 1 && cin >= 8 && cin % 8 == 0 && cin <= 65536 && cout >= 8 && cout % 8 == 0 &&
           cout <= 65536 && (ksize == 1 || ksize == 3) && int64_t(n) * h * wd <= INT32_MAX / 2;
}

}  // namespace

namespace {

// Scratch of the initial-field calls: two sets of three fp64 planes, then the non-finite count.
size_t fields_work_bytes(int64_t n) { return sizeof(double) * 6 * size_t(n) + sizeof(long long); }

lbm_status fields_check(const float* pred, int32_t stride, const uint8_t* solid, int32_t nx, int32_t ny,
                        int32_t smooth_iters, int32_t periodic, double u_scale, double rho_scale, double rho0,
                        const double* rho, const double* ux, const double* uy, const int64_t* n_bad)
{
    if (!pred || !solid || !rho || !ux || !uy || !n_bad) return fail(LBM_E_INVAL, "null argument");
    if (nx < 1 || ny < 1 || int64_t(nx) * ny > INT32_MAX / 8 || stride < 3 || smooth_iters < 0 ||
        smooth_iters > 1000 || (periodic != 0 && periodic != 1))
        return fail(LBM_E_INVAL, "arguments out of range");
    if (!std::isfinite(u_scale) || !std::isfinite(rho_scale) || !std::isfinite(rho0))
        return fail(LBM_E_INVAL, "non-finite scale");
    return LBM_OK;
}

// Unpack, smoothing passes and the fields, with the scratch at `work` (fields_work_bytes of n).
lbm_status fields_run(const float* pred, int32_t stride, const uint8_t* solid, int32_t nx, int32_t ny,
                      int32_t smooth_iters, int32_t periodic, double u_scale, double rho_scale, double rho0,
                      double* rho, double* ux, double* uy, int64_t* n_bad, void* work, hipStream_t st)
{
    const int n = nx * ny;
    double* t0 = static_cast<double*>(work);
    double* t1 = t0 + 3 * size_t(n);
    long long* d_bad = reinterpret_cast<long long*>(t1 + 3 * size_t(n));
    hipLaunchKernelGGL(lbm::nn::k_unpack, dim3(lbm::nn::blocks(size_t(n))), dim3(256), 0, st, pred, stride, solid, n,
                       t0);
    for (int i = 0; i < smooth_iters; ++i) {
        hipLaunchKernelGGL(lbm::nn::k_smooth, dim3(lbm::nn::blocks(size_t(n))), dim3(256), 0, st, t0, t1, solid, nx, ny,
                           periodic);
        std::swap(t0, t1);
    }
    // k_fields writes the count (it does not accumulate), so the scratch needs no clearing
    hipLaunchKernelGGL(lbm::nn::k_fields, dim3(1), dim3(1024), 0, st, t0, solid, n, u_scale, rho_scale, rho0, rho, ux,
                       uy, d_bad);
    long long h_bad = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&h_bad, d_bad, sizeof(long long), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(LBM_E_HIP, "initial fields: %s", hipGetErrorString(e));
    *n_bad = h_bad;
    return LBM_OK;
}

// Fixed scratch of lbm_nn_fields_noalloc: every GPU the library runs on holds its own copy for the
// life of the process.  Host code never uses the array's name as an address (on the host it is only
// a stand-in): fields_scratch() looks up the device address once per device, with that device
// current, and every later use goes through that address.
constexpr int64_t kFieldsScratchSites = int64_t(1) << 18;  // 512 x 512 sites, 12.6 MB
constexpr size_t kFieldsScratchWords = (6 * size_t(kFieldsScratchSites) * sizeof(double) + sizeof(long long) + 7) / 8;
__device__ __align__(256) double scratch[kFieldsScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

lbm_status fields_scratch(void** out)
{
    int dev = 0;
    LBM_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_E_INVAL, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LBM_E_HIP, "scratch address on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_conv2d_forward(const void* in, const void* w, const float* bias, void* out, float* out32, int32_t n,
                              int32_t h, int32_t wd, int32_t cin, int32_t cout, int32_t ksize, int32_t relu,
                              int32_t periodic, void* stream)
{
    if (!in || !w || (!out && !out32)) return fail(LBM_E_INVAL, "null argument");
    if (!conv_sizes_ok(n, h, wd, cin, cout, ksize)) return fail(LBM_E_INVAL, "convolution sizes out of range");
    if (!aligned16(in) || !aligned16(w) || (out && !aligned16(out)))
        return fail(LBM_E_INVAL, "bf16 tensors need 16-byte alignment");
    LBM_HIP_TRY(lbm::nn::conv_forward(cs(static_cast<const bf16*>(in), cin), static_cast<const bf16*>(w), bias,
                                      sl(static_cast<bf16*>(out), cout), out32, n, h, wd, cin, cout, ksize * ksize,
                                      relu != 0, periodic != 0, static_cast<hipStream_t>(stream), nullptr, 0));
    return LBM_OK;
}

lbm_status lbm_conv2d_dgrad(const void* dout, const void* w, void* din, void* wt, int32_t n, int32_t h, int32_t wd,
                            int32_t cin, int32_t cout, int32_t ksize, int32_t periodic, void* stream)
{
    if (!dout || !w || !din || !wt) return fail(LBM_E_INVAL, "null argument");
    if (!conv_sizes_ok(n, h, wd, cin, cout, ksize)) return fail(LBM_E_INVAL, "convolution sizes out of range");
    if (!aligned16(dout) || !aligned16(din) || !aligned16(wt)) return fail(LBM_E_INVAL, "bf16 tensors need 16-byte alignment");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int taps = ksize * ksize;
    LBM_HIP_TRY(lbm::nn::flip(static_cast<const bf16*>(w), static_cast<bf16*>(wt), taps, cout, cin, st));
    LBM_HIP_TRY(lbm::nn::conv_dgrad(cs(static_cast<const bf16*>(dout), cout), static_cast<const bf16*>(wt),
                                    sl(static_cast<bf16*>(din), cin), n, h, wd, cin, cout, taps, periodic != 0, st,
                                    nullptr, 0));
    return LBM_OK;
}

lbm_status lbm_conv2d_wgrad_workspace(int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout, int32_t ksize,
                                      int64_t* elems)
{
    if (!elems) return fail(LBM_E_INVAL, "null argument");
    if (!conv_sizes_ok(n, h, wd, cin, cout, ksize)) return fail(LBM_E_INVAL, "convolution sizes out of range");
    *elems = int64_t(lbm::nn::wgrad_plan(n, h, wd, cin, cout, ksize * ksize).elems);
    return LBM_OK;
}

lbm_status lbm_conv2d_wgrad(const void* in, const void* dout, float* dw, float* db, float* work, int64_t work_elems,
                            int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout, int32_t ksize, int32_t periodic,
                            void* stream)
{
    if (!in || !dout || !dw || !work) return fail(LBM_E_INVAL, "null argument");
    int64_t need = 0;
    const lbm_status s = lbm_conv2d_wgrad_workspace(n, h, wd, cin, cout, ksize, &need);
    if (s != LBM_OK) return s;
    if (work_elems < need)
        return fail(LBM_E_INVAL, "workspace too small (%lld < %lld)", (long long)work_elems, (long long)need);
    if (!aligned16(in) || !aligned16(dout)) return fail(LBM_E_INVAL, "bf16 tensors need 16-byte alignment");
    LBM_HIP_TRY(lbm::nn::conv_wgrad(cs(static_cast<const bf16*>(in), cin), cs(static_cast<const bf16*>(dout), cout),
                                    dw, db, work, n, h, wd, cin, cout, ksize * ksize, periodic != 0,
                                    static_cast<hipStream_t>(stream)));
    return LBM_OK;
}

lbm_status lbm_nn_create(const lbm_nn_config* cfg, uint64_t seed, void* stream, lbm_nn** out)
{
    if (!out || !cfg) return fail(LBM_E_INVAL, "null argument");
    *out = nullptr;
    const lbm_nn_config c = *cfg;
    if (c.levels < 1 || c.levels > 8 || c.base_channels < 8 || c.base_channels % 8 || c.in_channels < 1 ||
        c.in_channels > 4096 || c.out_channels < 1 || c.out_channels > kOutPad || c.max_batch < 1 || c.height < 1 ||
        c.width < 1 || (int64_t(c.base_channels) << (c.levels - 1)) > 8192)
        return fail(LBM_E_INVAL, "network configuration out of range");
    if (c.height % (1 << (c.levels - 1)) || c.width % (1 << (c.levels - 1)))
        return fail(LBM_E_INVAL, "height and width must be multiples of 2^(levels-1)");
    if (c.periodic != 0 && c.periodic != 1) return fail(LBM_E_INVAL, "periodic must be 0 or 1");
    if (int64_t(c.max_batch) * c.height * c.width > INT32_MAX / 8)
        return fail(LBM_E_INVAL, "max_batch * height * width too large");
    lbm_nn* n = new lbm_nn();
    n->cfg = c;
    n->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&n->device) != hipSuccess) {
        delete n;
        return fail(LBM_E_HIP, "no HIP device available");
    }
    const int L = c.levels;
    n->lv.resize(size_t(L));
    size_t off = 0;
    auto add = [&](Conv& cv, int taps, int cin, int cout, int level) {
        cv.taps = taps;
        cv.cin = cin;
        cv.cout = cout;
        cv.level = level;
        cv.w_off = off;
        off += size_t(taps) * cin * cout;
        cv.b_off = off;
        off += size_t(cout);
        n->convs.push_back(&cv);
    };
    for (int l = 0; l < L; ++l) {
        Level& v = n->lv[l];
        v.H = c.height >> l;
        v.W = c.width >> l;
        v.C = chan(n, l);
        v.cin = l == 0 ? (c.in_channels + 7) / 8 * 8 : chan(n, l - 1);
        add(v.c1, 9, v.cin, v.C, l);
        add(v.c2, 9, v.C, v.C, l);
    }
    for (int l = L - 2; l >= 0; --l) {
        Level& v = n->lv[l];
        add(v.d1, 9, chan(n, l + 1) + v.C, v.C, l);
        add(v.d2, 9, v.C, v.C, l);
    }
    add(n->out, 1, chan(n, 0), kOutPad, 0);
    n->n_params = off;
    const size_t B = size_t(c.max_batch);
    bool ok = nn_alloc(n, &n->w, off) && nn_alloc(n, &n->g, off) && nn_alloc(n, &n->m, off) &&
              nn_alloc(n, &n->v, off) && nn_alloc(n, &n->wb, off) && nn_alloc(n, &n->wt_all, off);
    size_t max_act = 0, work = 0;
    for (int l = 0; l < L && ok; ++l) {
        Level& v = n->lv[l];
        const size_t px = B * v.H * v.W;
        const int ccat = l < L - 1 ? chan(n, l + 1) + v.C : 0;
        max_act = std::max(max_act, px * size_t(v.C));
        ok = nn_alloc(n, &v.in, px * v.cin) && nn_alloc(n, &v.e1, px * v.C) && nn_alloc(n, &v.g_in, px * v.cin) &&
             nn_alloc(n, &v.g_e1, px * v.C);
        if (ok && l < L - 1)
            ok = nn_alloc(n, &v.cat, px * ccat) && nn_alloc(n, &v.g_cat, px * ccat) && nn_alloc(n, &v.d1o, px * v.C) &&
                 nn_alloc(n, &v.g_d1o, px * v.C) && nn_alloc(n, &v.d2o, px * v.C) && nn_alloc(n, &v.g_d2o, px * v.C);
        if (ok && l == L - 1) ok = nn_alloc(n, &v.e2, px * v.C) && nn_alloc(n, &v.g_e2, px * v.C);
    }
    for (const Conv* cv : n->convs) {
        // weight-gradient split partials, split-K partial sums of the forward and of the input
        // gradient (channel roles exchanged), for every batch size up to the maximum
        const int lh = n->lv[cv->level].H, lw = n->lv[cv->level].W;
        for (int nb = 1; nb <= int(B); ++nb) {
            work = std::max(work, lbm::nn::wgrad_plan(nb, lh, lw, cv->cin, cv->cout, cv->taps).elems);
            work = std::max(work, size_t(relu_bias_chunks(nb * lh * lw)) * size_t(cv->cout));
            work = std::max(work, lbm::nn::fwd_split_elems(nb, lh, lw, cv->cin, cv->cout, cv->taps));
            work = std::max(work, lbm::nn::fwd_split_elems(nb, lh, lw, cv->cout, cv->cin, cv->taps));
        }
    }
    n->work_elems = work;
    const size_t px0 = B * c.height * c.width;
    ok = ok && nn_alloc(n, &n->dz, max_act) && nn_alloc(n, &n->work, work) && nn_alloc(n, &n->part, px0 / 256 + 1) &&
         nn_alloc(n, &n->yout, px0 * kOutPad) && nn_alloc(n, &n->g_out, px0 * kOutPad) && nn_alloc(n, &n->d_red, 2) &&
         hipHostMalloc(reinterpret_cast<void**>(&n->h_red), 2 * sizeof(double), hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        nn_release(n);
        return fail(LBM_E_NOMEM, "network allocation failed");
    }
    for (Conv* cv : n->convs) {
        cv->w = n->wb + cv->w_off;
        cv->wt = n->wt_all + cv->w_off;
    }
    // seeded He-normal weights, zero biases; padded input and output channels start (and stay) 0
    std::vector<float> hp(off, 0.f);
    std::mt19937_64 rng(seed);
    for (const Conv* cv : n->convs) {
        std::normal_distribution<float> nd(0.f, std::sqrt(2.f / float(cv->taps * cv->cin)));
        for (int t = 0; t < cv->taps; ++t)
            for (int co = 0; co < cv->cout; ++co)
                for (int ci = 0; ci < cv->cin; ++ci) {
                    const float val = nd(rng);
                    const bool dead =
                        (cv == &n->out && co >= c.out_channels) || (cv == &n->lv[0].c1 && ci >= c.in_channels);
                    hp[cv->w_off + (size_t(t) * cv->cout + co) * cv->cin + ci] = dead ? 0.f : val;
                }
    }
    const lbm_status st = lbm_nn_set_params(n, hp.data());
    if (st != LBM_OK) {
        nn_release(n);
        return st;
    }
    *out = n;
    return LBM_OK;
}

lbm_status lbm_nn_destroy(lbm_nn* n)
{
    nn_release(n);
    return LBM_OK;
}

lbm_status lbm_nn_param_count(const lbm_nn* n, int64_t* count)
{
    if (!n || !count) return fail(LBM_E_INVAL, "null argument");
    *count = int64_t(n->n_params);
    return LBM_OK;
}

lbm_status lbm_nn_set_params(lbm_nn* n, const float* host)
{
    if (!n || !host) return fail(LBM_E_INVAL, "null argument");
    DeviceGuard g(n->device);
    LBM_HIP_TRY(hipMemcpyAsync(n->w, host, sizeof(float) * n->n_params, hipMemcpyHostToDevice, n->stream));
    LBM_HIP_TRY(lbm::launch_fill_zero(n->m, sizeof(float) * n->n_params, n->stream));
    LBM_HIP_TRY(lbm::launch_fill_zero(n->v, sizeof(float) * n->n_params, n->stream));
    LBM_HIP_TRY(lbm::launch_fill_zero(n->g, sizeof(float) * n->n_params, n->stream));
    hipLaunchKernelGGL(lbm::nn::k_to_bf16, dim3(lbm::nn::blocks(n->n_params)), dim3(256), 0, n->stream, n->w, n->wb,
                       n->n_params);
    LBM_HIP_TRY(hipGetLastError());
    LBM_HIP_TRY(refresh_flipped(n));
    LBM_HIP_TRY(hipStreamSynchronize(n->stream));
    n->adam_t = 0;
    return LBM_OK;
}

lbm_status lbm_nn_get_params(const lbm_nn* n, float* host)
{
    if (!n || !host) return fail(LBM_E_INVAL, "null argument");
    DeviceGuard g(n->device);
    LBM_HIP_TRY(hipMemcpyAsync(host, n->w, sizeof(float) * n->n_params, hipMemcpyDeviceToHost, n->stream));
    LBM_HIP_TRY(hipStreamSynchronize(n->stream));
    return LBM_OK;
}

lbm_status lbm_nn_get_grads(const lbm_nn* n, float* host)
{
    if (!n || !host) return fail(LBM_E_INVAL, "null argument");
    DeviceGuard g(n->device);
    LBM_HIP_TRY(hipMemcpyAsync(host, n->g, sizeof(float) * n->n_params, hipMemcpyDeviceToHost, n->stream));
    LBM_HIP_TRY(hipStreamSynchronize(n->stream));
    return LBM_OK;
}

lbm_status lbm_nn_forward(lbm_nn* n, const void* x, float* y, int32_t batch)
{
    if (!n || !x) return fail(LBM_E_INVAL, "null argument");
    if (batch < 1 || batch > n->cfg.max_batch) return fail(LBM_E_INVAL, "batch outside 1 .. max_batch");
    if (!aligned16(x)) return fail(LBM_E_INVAL, "input needs 16-byte alignment");
    DeviceGuard g(n->device);
    const int L = n->cfg.levels, N = batch;
    Level& v0 = n->lv[0];
    LBM_HIP_TRY(hipMemcpyAsync(v0.in, x, sizeof(bf16) * size_t(N) * v0.H * v0.W * v0.cin, hipMemcpyDeviceToDevice,
                               n->stream));
    for (int l = 0; l < L; ++l) {  // encoder
        Level& v = n->lv[l];
        LBM_HIP_TRY(fwd(n, v.c1, cs(v.in, v.cin), sl(v.e1, v.C), nullptr, N, v.H, v.W, true));
        // the second convolution writes the skip slice of the concatenation and the pooled input of
        // the level below
        const Slice skip = l < L - 1 ? sl(v.cat, chan(n, l + 1) + v.C, chan(n, l + 1)) : sl(v.e2, v.C);
        const Slice pooled = l < L - 1 ? sl(n->lv[l + 1].in, v.C) : Slice{nullptr, 0, 0};
        LBM_HIP_TRY(fwd(n, v.c2, cs(v.e1, v.C), skip, nullptr, N, v.H, v.W, true, pooled));
    }
    for (int l = L - 2; l >= 0; --l) {  // decoder
        Level& v = n->lv[l];
        const Level& below = n->lv[l + 1];
        const int cup = chan(n, l + 1), ccat = cup + v.C;
        // the first convolution reads the upsampled part of its input straight from the level below
        // (written into the concatenation only where a kernel needs it there)
        const lbm::nn::UpSrc up{l == L - 2 ? cs(below.e2, below.C) : cs(below.d2o, below.C), cup, sl(v.cat, ccat, 0)};
        LBM_HIP_TRY(fwd(n, v.d1, cs(v.cat, ccat), sl(v.d1o, v.C), nullptr, N, v.H, v.W, true, Slice{nullptr, 0, 0},
                        lbm::nn::Out1{nullptr, nullptr, nullptr, 0}, up));
        // level 0: the output 1x1 convolution follows the last 3x3 one
        const lbm::nn::Out1 o1 = l == 0 ? lbm::nn::Out1{n->out.w, n->w + n->out.b_off, n->yout, kOutPad}
                                        : lbm::nn::Out1{nullptr, nullptr, nullptr, 0};
        LBM_HIP_TRY(fwd(n, v.d2, cs(v.d1o, v.C), sl(v.d2o, v.C), nullptr, N, v.H, v.W, true, Slice{nullptr, 0, 0}, o1));
    }
    if (L == 1) LBM_HIP_TRY(fwd(n, n->out, cs(v0.e2, v0.C), Slice{nullptr, 0, 0}, n->yout, N, v0.H, v0.W, false));
    n->last_n = N;
    if (y) {
        const int oc = n->cfg.out_channels;
        LBM_HIP_TRY(hipMemcpy2DAsync(y, sizeof(float) * oc, n->yout, sizeof(float) * kOutPad, sizeof(float) * oc,
                                     size_t(N) * v0.H * v0.W, hipMemcpyDeviceToDevice, n->stream));
    }
    return LBM_OK;
}

lbm_status lbm_nn_backward(lbm_nn* n, const float* target, const uint8_t* mask, int32_t batch, double* loss)
{
    if (!n || !target || !mask) return fail(LBM_E_INVAL, "null argument");
    if (batch != n->last_n || batch < 1) return fail(LBM_E_STATE, "backward needs the batch of the last forward");
    DeviceGuard g(n->device);
    const int L = n->cfg.levels, N = batch;
    Level& v0 = n->lv[0];
    const int P0 = N * v0.H * v0.W, oc = n->cfg.out_channels, nb = (P0 + 255) / 256;
    // loss over fluid pixels and the gradient of the output
    hipLaunchKernelGGL(lbm::nn::k_mask_count, dim3(nb), dim3(256), 0, n->stream, mask, P0, n->part);
    hipLaunchKernelGGL(lbm::nn::k_sum_partials, dim3(1), dim3(256), 0, n->stream, n->part, nb, n->d_red);
    hipLaunchKernelGGL(lbm::nn::k_mse, dim3(nb), dim3(256), 0, n->stream, n->yout, target, mask, P0, kOutPad, oc,
                       n->d_red, n->g_out, n->part);
    hipLaunchKernelGGL(lbm::nn::k_sum_partials, dim3(1), dim3(256), 0, n->stream, n->part, nb, n->d_red + 1);
    LBM_HIP_TRY(hipGetLastError());
    LBM_HIP_TRY(hipMemcpyAsync(n->h_red, n->d_red, 2 * sizeof(double), hipMemcpyDeviceToHost, n->stream));
    // 1x1 output convolution (no activation)
    const CSlice top = L == 1 ? cs(v0.e2, v0.C) : cs(v0.d2o, v0.C);
    const Slice g_top = L == 1 ? sl(v0.g_e2, v0.C) : sl(v0.g_d2o, v0.C);
    LBM_HIP_TRY(wgrad(n, n->out, top, cs(n->g_out, kOutPad), N, v0.H, v0.W));
    LBM_HIP_TRY(lbm::nn::conv_dgrad(cs(n->g_out, kOutPad), n->out.wt, g_top, N, v0.H, v0.W, n->out.cin, n->out.cout,
                                    1, false, n->stream, n->work, n->work_elems));
    // decoder, level 0 up to the level above the bottleneck
    for (int l = 0; l <= L - 2; ++l) {
        Level& v = n->lv[l];
        Level& below = n->lv[l + 1];
        const int cup = chan(n, l + 1), ccat = cup + v.C;
        LBM_HIP_TRY(conv_relu_bwd(n, v.d2, cs(v.d1o, v.C), cs(v.d2o, v.C), cs(v.g_d2o, v.C), sl(v.g_d1o, v.C), N, v.H,
                                  v.W));
        const lbm::nn::UpSrc up{l == L - 2 ? cs(below.e2, below.C) : cs(below.d2o, below.C), cup, sl(v.cat, ccat, 0)};
        LBM_HIP_TRY(conv_relu_bwd(n, v.d1, cs(v.cat, ccat), cs(v.d1o, v.C), cs(v.g_d1o, v.C), sl(v.g_cat, ccat), N,
                                  v.H, v.W, up));
        // upsampled part of the concatenation -> gradient of the level below's output
        const Slice gsrc = l == L - 2 ? sl(below.g_e2, below.C) : sl(below.g_d2o, below.C);
        hipLaunchKernelGGL(lbm::nn::k_up_bwd, dim3(lbm::nn::blocks(size_t(N) * below.H * below.W * cup / 8)), dim3(256),
                           0, n->stream, cs(v.g_cat, ccat, 0), gsrc, N, below.H, below.W, cup);
        LBM_HIP_TRY(hipGetLastError());
    }
    // encoder, bottleneck down to level 0; the skip gradients already sit in the concatenation
    // gradients, and the pooling gradients are added to them on the way
    for (int l = L - 1; l >= 0; --l) {
        Level& v = n->lv[l];
        const int cup = l < L - 1 ? chan(n, l + 1) : 0;
        const CSlice y2 = l < L - 1 ? cs(v.cat, cup + v.C, cup) : cs(v.e2, v.C);
        const CSlice g2 = l < L - 1 ? cs(v.g_cat, cup + v.C, cup) : cs(v.g_e2, v.C);
        LBM_HIP_TRY(conv_relu_bwd(n, v.c2, cs(v.e1, v.C), y2, g2, sl(v.g_e1, v.C), N, v.H, v.W));
        const Slice gin = l > 0 ? sl(v.g_in, v.cin) : Slice{nullptr, 0, 0};
        LBM_HIP_TRY(conv_relu_bwd(n, v.c1, cs(v.in, v.cin), cs(v.e1, v.C), cs(v.g_e1, v.C), gin, N, v.H, v.W));
        if (l > 0) {
            Level& up = n->lv[l - 1];
            const Slice g_skip = sl(up.g_cat, chan(n, l) + up.C, chan(n, l));
            hipLaunchKernelGGL(lbm::nn::k_pool_bwd_add, dim3(lbm::nn::blocks(size_t(N) * up.H * up.W * up.C / 8)),
                               dim3(256), 0, n->stream, cs(v.g_in, v.cin), g_skip, N, up.H, up.W, up.C);
            LBM_HIP_TRY(hipGetLastError());
        }
    }
    LBM_HIP_TRY(hipStreamSynchronize(n->stream));
    if (loss) *loss = n->h_red[1] / (std::max(n->h_red[0], 1.0) * oc);
    return LBM_OK;
}

lbm_status lbm_nn_adam_step(lbm_nn* n, float lr, float beta1, float beta2, float eps)
{
    if (!n) return fail(LBM_E_INVAL, "null network");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(LBM_E_INVAL, "Adam hyper-parameters out of range");
    DeviceGuard g(n->device);
    n->adam_t += 1;
    const float c1 = 1.f - std::pow(beta1, float(n->adam_t)), c2 = 1.f - std::pow(beta2, float(n->adam_t));
    hipLaunchKernelGGL(lbm::nn::k_adam, dim3(lbm::nn::blocks(n->n_params)), dim3(256), 0, n->stream, n->w, n->m, n->v,
                       n->g, n->wb, n->n_params, lr, beta1, beta2, eps, c1, c2);
    LBM_HIP_TRY(hipGetLastError());
    LBM_HIP_TRY(refresh_flipped(n));
    return LBM_OK;
}

lbm_status lbm_nn_features(const uint8_t* solid, const lbm_link* links, int64_t n_links, int32_t nx, int32_t ny,
                           float kn_feature, float ax_feature, float ay_feature, void* out, int32_t channels,
                           void* stream)
{
    if (!solid || !out || (n_links > 0 && !links)) return fail(LBM_E_INVAL, "null argument");
    if (nx < 1 || ny < 1 || int64_t(nx) * ny > INT32_MAX / 64 || n_links < 0 || channels < 16 || channels % 8 ||
        channels > 4096)
        return fail(LBM_E_INVAL, "feature sizes out of range");
    if (!aligned16(out)) return fail(LBM_E_INVAL, "output needs 16-byte alignment");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int n = nx * ny;
    bf16* x = static_cast<bf16*>(out);
    hipLaunchKernelGGL(lbm::nn::k_feat_sites, dim3(lbm::nn::blocks(size_t(n))), dim3(256), 0, st, solid, n, kn_feature,
                       ax_feature, ay_feature, x, channels);
    if (n_links > 0)
        hipLaunchKernelGGL(lbm::nn::k_feat_links, dim3(lbm::nn::blocks(size_t(n_links))), dim3(256), 0, st, links,
                           n_links, solid, nx, ny, x, channels);
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_nn_fields(const float* pred, int32_t stride, const uint8_t* solid, int32_t nx, int32_t ny,
                         int32_t smooth_iters, int32_t periodic, double u_scale, double rho_scale, double rho0,
                         double* rho, double* ux, double* uy, int64_t* n_bad, void* stream)
{
    lbm_status st = fields_check(pred, stride, solid, nx, ny, smooth_iters, periodic, u_scale, rho_scale, rho0, rho,
                                 ux, uy, n_bad);
    if (st != LBM_OK) return st;
    void* work = nullptr;
    LBM_HIP_TRY(hipMalloc(&work, fields_work_bytes(int64_t(nx) * ny)));
    st = fields_run(pred, stride, solid, nx, ny, smooth_iters, periodic, u_scale, rho_scale, rho0, rho, ux, uy, n_bad,
                    work, static_cast<hipStream_t>(stream));
    ignore(hipFree(work));
    return st;
}

lbm_status lbm_nn_fields_noalloc(const float* pred, int32_t stride, const uint8_t* solid, int32_t nx, int32_t ny,
                                 int32_t smooth_iters, int32_t periodic, double u_scale, double rho_scale,
                                 double rho0, double* rho, double* ux, double* uy, int64_t* n_bad, void* stream)
{
    lbm_status st = fields_check(pred, stride, solid, nx, ny, smooth_iters, periodic, u_scale, rho_scale, rho0, rho,
                                 ux, uy, n_bad);
    if (st != LBM_OK) return st;
    if (int64_t(nx) * ny > kFieldsScratchSites)
        return fail(LBM_E_INVAL, "lbm_nn_fields_noalloc: %d x %d sites exceed its fixed scratch of %lld sites", nx,
                    ny, (long long)kFieldsScratchSites);
    void* work = nullptr;
    st = fields_scratch(&work);
    if (st != LBM_OK) return st;
    return fields_run(pred, stride, solid, nx, ny, smooth_iters, periodic, u_scale, rho_scale, rho0, rho, ux, uy,
                      n_bad, work, static_cast<hipStream_t>(stream));
}

}  // extern "C"
