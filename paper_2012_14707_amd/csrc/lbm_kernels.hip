// HIP kernels of liblbm for gfx950 (CDNA4, 64-wide wavefronts).
//
// Storage: populations as deviations g_i = f_i - w_i rho0 from the rest equilibrium, in nine
// planes (structure of arrays) of n sites each, "pull" layout: plane i at site y holds the value
// that site y + c_i receives at the next time level.  A fluid site therefore reads its nine
// incoming populations at x - c_i (one coalesced, possibly one-element-shifted, load per plane)
// and writes its nine outgoing values at its own index (fully coalesced).  For a wall link
// (x, ibar) the incoming population i comes from the solid site x + c_ibar; the boundary rule of
// Eq. (EqNewBDSC) writes it there, a slot no other site writes.
//
// The kernels are bound by HBM traffic (about 1-2 flop per byte); the 9x9 moment transform is
// applied in closed form with additions only, not as a dense contraction.
#include <hip/hip_runtime.h>

#include "lbm_internal.hpp"

namespace lbm {
namespace {

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

// Exclusive prefix over the wavefront of a per-lane count in [0, 15].
__device__ __forceinline__ uint32_t wave_prefix4(uint32_t v)
{
    const uint64_t b0 = __ballot(v & 1u);
    const uint64_t b1 = __ballot(v & 2u);
    const uint64_t b2 = __ballot(v & 4u);
    const uint64_t b3 = __ballot(v & 8u);
    return lanes_below(b0) + 2u * lanes_below(b1) + 4u * lanes_below(b2) + 8u * lanes_below(b3);
}

struct Nbr {
    uint32_t x, xm, xp, row, rowm, rowp;
};

__device__ __forceinline__ Nbr neighbours(uint32_t s, uint32_t nx, uint32_t ny)
{
    Nbr b;
    const uint32_t y = s / nx;
    b.x = s - y * nx;
    b.xm = (b.x == 0u) ? nx - 1u : b.x - 1u;
    b.xp = (b.x + 1u == nx) ? 0u : b.x + 1u;
    const uint32_t ym = (y == 0u) ? ny - 1u : y - 1u;
    const uint32_t yp = (y + 1u == ny) ? 0u : y + 1u;
    b.row = y * nx;
    b.rowm = ym * nx;
    b.rowp = yp * nx;
    return b;
}

// 1/9 and 1/6 as an unevaluated sum hi + lo of two values of the storage type.
template <typename T>
struct Third;
template <>
struct Third<double> {
    static constexpr double c9_hi = 1.0 / 9.0;
    static constexpr double c9_lo = 6.1679056923619804e-18;   // 1/9 - c9_hi, evaluated exactly
    static constexpr double c6_hi = 1.0 / 6.0;
    static constexpr double c6_lo = 9.2518585385429707e-18;   // 1/6 - c6_hi, evaluated exactly
};
template <>
struct Third<float> {
    static constexpr float c9_hi = 1.0f / 9.0f;
    static constexpr float c9_lo = static_cast<float>(1.0 / 9.0 - static_cast<double>(1.0f / 9.0f));
    static constexpr float c6_hi = 1.0f / 6.0f;
    static constexpr float c6_lo = static_cast<float>(1.0 / 6.0 - static_cast<double>(1.0f / 6.0f));
};

template <typename T>
__device__ __forceinline__ T split_mul(T x, T hi, T lo) { return fma(x, hi, x * lo); }

// The nine pulled populations g_i(x, t) (D2Q9 order of Eq. (Eq3)).
template <typename T>
struct Pop {
    T g0, g1, g2, g3, g4, g5, g6, g7, g8;
};

template <typename T>
__device__ __forceinline__ Pop<T> pull(const T* __restrict__ src, uint64_t n, uint32_t s, const Nbr& b)
{
    Pop<T> p;
    p.g0 = src[s];
    p.g1 = src[1 * n + b.row + b.xm];   // from (x-1, y)
    p.g2 = src[2 * n + b.rowm + b.x];   // from (x, y-1)
    p.g3 = src[3 * n + b.row + b.xp];   // from (x+1, y)
    p.g4 = src[4 * n + b.rowp + b.x];   // from (x, y+1)
    p.g5 = src[5 * n + b.rowm + b.xm];  // from (x-1, y-1)
    p.g6 = src[6 * n + b.rowm + b.xp];  // from (x+1, y-1)
    p.g7 = src[7 * n + b.rowp + b.xp];  // from (x+1, y+1)
    p.g8 = src[8 * n + b.rowp + b.xm];  // from (x-1, y+1)
    return p;
}

// Density deviation and half-force velocity (Eq. (FluidMacr)) accumulated in fp64, for the
// residual, the recorded velocity and the moments output.
template <typename T>
__device__ __forceinline__ void macro_fp64(const Pop<T>& p, double rho0, double ax, double ay, double& dr,
                                           double& rho, double& ux, double& uy)
{
    const double g0 = p.g0, g1 = p.g1, g2 = p.g2, g3 = p.g3, g4 = p.g4, g5 = p.g5, g6 = p.g6, g7 = p.g7,
                 g8 = p.g8;
    dr = (g0 + ((g1 + g2) + (g3 + g4))) + ((g5 + g6) + (g7 + g8));
    rho = rho0 + dr;
    const double jx = (g1 - g3) + (g5 - g6) + (g8 - g7);
    const double jy = (g2 - g4) + (g5 + g6) - (g7 + g8);
    ux = (jx + 0.5 * rho * ax) / rho;
    uy = (jy + 0.5 * rho * ay) / rho;
}

// One boundary value of Eq. (EqNewBDSC) in deviation form (see the header of this file):
//   g_i(x_f, t+1) = a1 g_ibar + a2 g'_i + a3 g'_ibar + beta rho + kappa w_i (drho + rho phi_i(u)),
// phi_i(u) = 3 c_i.u + 4.5 (c_i.u)^2 - 1.5 u^2, and the rho phi term only in the node reading.
template <typename T, bool NODE>
__device__ __forceinline__ T boundary_value(const LinkCoef<T>& c, uint32_t k, T g_ibar, T h_i, T h_ibar, T rho,
                                            T dr, T w, T cu, T u2)
{
    T diffuse = dr;
    if (NODE) diffuse += rho * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * u2);
    return c.a1[k] * g_ibar + c.a2[k] * h_i + c.a3[k] * h_ibar + c.beta[k] * rho + c.kappa[k] * (w * diffuse);
}

template <typename T, bool WRITE_U, bool NODE, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_step(const StepArgs<T> a)
{
    uint32_t blk = blockIdx.x;
    if (blk < a.remap_blocks) blk = (blk & 7u) * (a.remap_blocks >> 3) + (blk >> 3);
    const uint32_t s = blk * BLOCK + threadIdx.x;
    const uint64_t n = a.n;
    const uint32_t fl = (s < a.n) ? static_cast<uint32_t>(a.flags[s]) : kSolid;
    const bool fluid = fl != kSolid;
    const uint32_t nlink = fluid ? static_cast<uint32_t>(__popc(fl)) : 0u;
    const uint32_t pre = wave_prefix4(nlink);  // every lane of the wave takes part
    if (!fluid) return;

    const Nbr b = neighbours(s, a.nx, a.ny);
    const Pop<T> p = pull(a.src, n, s, b);
    const T g0 = p.g0, g1 = p.g1, g2 = p.g2, g3 = p.g3, g4 = p.g4, g5 = p.g5, g6 = p.g6, g7 = p.g7, g8 = p.g8;

    if (WRITE_U) {
        double dr_d, rho_d, ux_d, uy_d;
        macro_fp64(p, static_cast<double>(a.rho0), static_cast<double>(a.ax), static_cast<double>(a.ay), dr_d,
                   rho_d, ux_d, uy_d);
        a.ux_out[s] = ux_d;
        a.uy_out[s] = uy_d;
    }

    // conserved moments and half-force velocity, Eq. (FluidMacr)
    const T s14 = (g1 + g2) + (g3 + g4);
    const T s58 = (g5 + g6) + (g7 + g8);
    const T dr = g0 + s14 + s58;
    const T rho = a.rho0 + dr;
    const T jx = (g1 - g3) + (g5 - g6) + (g8 - g7);
    const T jy = (g2 - g4) + (g5 + g6) - (g7 + g8);
    const T irho = T(1) / rho;
    const T ux = (jx + T(0.5) * rho * a.ax) * irho;
    const T uy = (jy + T(0.5) * rho * a.ay) * irho;
    const T u2 = ux * ux + uy * uy;

    // non-conserved moments m = M g (rows of M in Sec. II)
    const T e = T(-4) * g0 - s14 + T(2) * s58;
    const T eps = T(4) * g0 - T(2) * s14 + s58;
    const T qx = T(-2) * (g1 - g3) + ((g5 - g6) + (g8 - g7));
    const T qy = T(-2) * (g2 - g4) + ((g5 + g6) - (g7 + g8));
    const T pxx = (g1 + g3) - (g2 + g4);
    const T pxy = (g5 + g7) - (g6 + g8);

    // equilibria of Eq. (LBEequi) in moment space (deviation from the rest state) and the Guo
    // forcing moments M Fbar of Eq. (LBEforce): (0, 6 rho u.a, -6 rho u.a, rho a_x, -rho a_x,
    // rho a_y, -rho a_y, 2 rho (u_x a_x - u_y a_y), rho (u_x a_y + u_y a_x))
    const T ru2 = T(3) * rho * u2;
    const T ua6 = T(6) * rho * (ux * a.ax + uy * a.ay);
    const T ep = e - a.s_e * (e - (T(-2) * dr + ru2)) + a.c_e * ua6;
    const T epsp = eps - a.s_eps * (eps - (dr - ru2)) - a.c_eps * ua6;
    const T qxp = qx - a.s_q * (qx + rho * ux) - a.c_q * (rho * a.ax);
    const T qyp = qy - a.s_q * (qy + rho * uy) - a.c_q * (rho * a.ay);
    const T pxxp = pxx - a.s_s * (pxx - rho * (ux * ux - uy * uy)) + a.c_s * (T(2) * rho * (ux * a.ax - uy * a.ay));
    const T pxyp = pxy - a.s_s * (pxy - rho * (ux * uy)) + a.c_s * (rho * (ux * a.ay + uy * a.ax));
    // conserved: rho' = rho; j' = j + rho a exactly (the tau_j relaxation and forcing cancel)
    const T jxp = jx + rho * a.ax;
    const T jyp = jy + rho * a.ay;

    // f' = M^-1 m' with M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
    // The conserved moments (rho, j) never relax, so a rounded constant 1/9 or 1/6 would scale
    // mass and momentum by (1 + its rounding error) at every collision and the bias would grow
    // over the whole run; they are divided with a two-term constant (error below one ulp, unbiased).
    const T r0 = split_mul(dr, Third<T>::c9_hi, Third<T>::c9_lo);
    const T r1 = ep * T(1.0 / 36.0);
    const T r2 = epsp * T(1.0 / 36.0);
    const T r3 = split_mul(jxp, Third<T>::c6_hi, Third<T>::c6_lo);
    const T r4 = qxp * T(1.0 / 12.0);
    const T r5 = split_mul(jyp, Third<T>::c6_hi, Third<T>::c6_lo);
    const T r6 = qyp * T(1.0 / 12.0);
    const T r7 = pxxp * T(0.25);
    const T r8 = pxyp * T(0.25);
    const T A = r0 - r1 - T(2) * r2;
    const T B = r0 + T(2) * r1 + r2;
    const T X = r3 - T(2) * r4, Y = r5 - T(2) * r6;
    const T XD = r3 + r4, YD = r5 + r6;
    const T h0 = r0 - T(4) * r1 + T(4) * r2;
    const T h1 = A + X + r7;
    const T h2 = A + Y - r7;
    const T h3 = A - X + r7;
    const T h4 = A - Y - r7;
    const T h5 = B + XD + YD + r8;
    const T h6 = B - XD + YD - r8;
    const T h7 = B - XD - YD + r8;
    const T h8 = B + XD - YD - r8;

    T* __restrict__ dst = a.dst;
    // Post-collision values leave along c_i and are pulled by x + c_i next step; the ones that
    // would enter a solid site are not needed and are not stored.
    dst[s] = h0;
    if (!(fl & 0x01u)) dst[1 * n + s] = h1;
    if (!(fl & 0x02u)) dst[2 * n + s] = h2;
    if (!(fl & 0x04u)) dst[3 * n + s] = h3;
    if (!(fl & 0x08u)) dst[4 * n + s] = h4;
    if (!(fl & 0x10u)) dst[5 * n + s] = h5;
    if (!(fl & 0x20u)) dst[6 * n + s] = h6;
    if (!(fl & 0x40u)) dst[7 * n + s] = h7;
    if (!(fl & 0x80u)) dst[8 * n + s] = h8;

    if (fl) {
        // wall links of this node, in direction order; link d (toward the wall) fills the unknown
        // i = opposite(d) at the solid site x + c_d
        uint32_t k = static_cast<uint32_t>(a.chunk_base[s / kChunk]) + pre;
        const T w1 = T(1.0 / 9.0), w5 = T(1.0 / 36.0);
        const LinkCoef<T> c = a.coef;
        if (fl & 0x01u) {  // d = 1 (E), unknown i = 3 (W): c_i.u = -ux
            dst[3 * n + b.row + b.xp] = boundary_value<T, NODE>(c, k, g1, h3, h1, rho, dr, w1, -ux, u2);
            ++k;
        }
        if (fl & 0x02u) {  // d = 2 (N), i = 4 (S)
            dst[4 * n + b.rowp + b.x] = boundary_value<T, NODE>(c, k, g2, h4, h2, rho, dr, w1, -uy, u2);
            ++k;
        }
        if (fl & 0x04u) {  // d = 3 (W), i = 1 (E)
            dst[1 * n + b.row + b.xm] = boundary_value<T, NODE>(c, k, g3, h1, h3, rho, dr, w1, ux, u2);
            ++k;
        }
        if (fl & 0x08u) {  // d = 4 (S), i = 2 (N)
            dst[2 * n + b.rowm + b.x] = boundary_value<T, NODE>(c, k, g4, h2, h4, rho, dr, w1, uy, u2);
            ++k;
        }
        if (fl & 0x10u) {  // d = 5 (NE), i = 7 (SW)
            dst[7 * n + b.rowp + b.xp] = boundary_value<T, NODE>(c, k, g5, h7, h5, rho, dr, w5, -ux - uy, u2);
            ++k;
        }
        if (fl & 0x20u) {  // d = 6 (NW), i = 8 (SE)
            dst[8 * n + b.rowp + b.xm] = boundary_value<T, NODE>(c, k, g6, h8, h6, rho, dr, w5, ux - uy, u2);
            ++k;
        }
        if (fl & 0x40u) {  // d = 7 (SW), i = 5 (NE)
            dst[5 * n + b.rowm + b.xm] = boundary_value<T, NODE>(c, k, g7, h5, h7, rho, dr, w5, ux + uy, u2);
            ++k;
        }
        if (fl & 0x80u) {  // d = 8 (SE), i = 6 (NW)
            dst[6 * n + b.rowm + b.xp] = boundary_value<T, NODE>(c, k, g8, h6, h8, rho, dr, w5, -ux + uy, u2);
        }
    }
}

// ------------------------------------------------------------------- per-link precompute

__device__ __forceinline__ double weight_of(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }

// Coefficients of Eq. (EqNewBDSC) per link from gamma, the l and r rules of Sec. III.B and the
// wall velocity; one thread per link, fp64.  Output rows of coef64 (n_links each):
// l_raw, l_eff, r, alpha1, alpha2, alpha3, beta, kappa.
__global__ void __launch_bounds__(256) k_precompute(const LinkInput in, const PrecomputeArgs a, double* coef64,
                                                    float* coef32)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= a.n_links) return;
    const int64_t nl = a.n_links;
    const double g = in.q[k];
    const double ts = a.tau_s, L1 = a.L1, E = a.E, sq = a.sq6pi;
    const double t2 = 2.0 * ts - 1.0;
    double l_raw;
    switch (a.l_mode) {
    case 2: l_raw = 0.0; break;
    case 3: l_raw = g; break;
    case 4: l_raw = 2.0 * g; break;
    case 5: l_raw = g * g; break;
    case 6: l_raw = g * g + g; break;
    case 7: l_raw = a.l_override; break;
    default: l_raw = (sq * g * g + g * t2 * (L1 + sq)) / (sq * t2) + E; break;  // Eq. (Eqexlva)
    }
    double l = l_raw;
    if (a.l_mode == 0 && l_raw < -0.4) l = 0.0;
    if (a.l_mode == 1 && l_raw < 0.0) l = 0.0;
    double r;
    if (a.r_mode == 2) {
        r = a.r_override;
    } else if (a.r_mode == 1) {  // Eq. (NSliCoertsr)
        const double br = g * g + g * t2 + (1.0 + E) * t2;
        r = (L1 * ts * g * t2 + sq * ts * br) / (L1 * t2 * ((2.0 + g) * ts - 1.0) + sq * ts * br);
    } else {  // Eq. (SliCoeffrtsr)
        r = sq * ts * (1.0 + l) / (L1 * t2 + sq * ts * (1.0 + l));
    }
    const int d = in.dir[k];
    const int i = (d <= 4) ? ((d + 1) & 3) + 1 : ((d - 3) & 3) + 5;  // opposite direction
    const int cxi = (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
    const int cyi = (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
    const double w = weight_of(i);
    const double inv = 1.0 / (1.0 + l);
    const double a1 = r * (1.0 + l - 2.0 * g) * inv;
    const double a2 = r * l * inv;
    const double a3 = r * (2.0 * g - l) * inv;
    const double cub = cxi * in.ubx[k] + cyi * in.uby[k];
    const double kappa = 1.0 - r;
    double beta = 2.0 * r * inv * w * 3.0 * cub;
    if (a.diffuse == 1) {
        const double ub2 = in.ubx[k] * in.ubx[k] + in.uby[k] * in.uby[k];
        beta += kappa * w * (3.0 * cub + 4.5 * cub * cub - 1.5 * ub2);
    }
    coef64[0 * nl + k] = l_raw;
    coef64[1 * nl + k] = l;
    coef64[2 * nl + k] = r;
    coef64[3 * nl + k] = a1;
    coef64[4 * nl + k] = a2;
    coef64[5 * nl + k] = a3;
    coef64[6 * nl + k] = beta;
    coef64[7 * nl + k] = kappa;
    // The deviation form of the step kernel uses a1 + a2 + a3 + kappa = 1 analytically (it never
    // forms w_i rho0 (a1 + a2 + a3 + kappa - 1)), so rounding the coefficients only perturbs their
    // products with the small deviations.
    if (coef32) {
        coef32[0 * nl + k] = static_cast<float>(a1);
        coef32[1 * nl + k] = static_cast<float>(a2);
        coef32[2 * nl + k] = static_cast<float>(a3);
        coef32[3 * nl + k] = static_cast<float>(beta);
        coef32[4 * nl + k] = static_cast<float>(kappa);
    }
}

// ------------------------------------------------------------------ init, moments, residual

__global__ void __launch_bounds__(256) k_fill_zero(uint4* p, uint64_t n16)
{
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n16) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void __launch_bounds__(256) k_fill_zero_bytes(uint8_t* p, uint64_t n)
{
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// f_i(x, 0) = f_i^eq(rho, u - a/2): stored at slot (i, x - c_i) as the deviation
// w_i (rho - rho0) + w_i rho (3 c.v + 4.5 (c.v)^2 - 1.5 v^2), v = u - a/2.
template <typename T>
__global__ void __launch_bounds__(256) k_init_fields(T* dst, const uint8_t* flags, const double* rho_in,
                                                     const double* ux_in, const double* uy_in, uint32_t n,
                                                     uint32_t nx, uint32_t ny, double rho0, double ax, double ay)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n || flags[s] == kSolid) return;
    const Nbr b = neighbours(s, nx, ny);
    const double rho = rho_in[s];
    const double vx = ux_in[s] - 0.5 * ax, vy = uy_in[s] - 0.5 * ay;
    const double v2 = vx * vx + vy * vy;
    const uint64_t N = n;
    auto dev = [&](double w, double cv) {
        return static_cast<T>(w * (rho - rho0) + w * rho * (3.0 * cv + 4.5 * cv * cv - 1.5 * v2));
    };
    dst[s] = dev(4.0 / 9.0, 0.0);
    dst[1 * N + b.row + b.xm] = dev(1.0 / 9.0, vx);
    dst[2 * N + b.rowm + b.x] = dev(1.0 / 9.0, vy);
    dst[3 * N + b.row + b.xp] = dev(1.0 / 9.0, -vx);
    dst[4 * N + b.rowp + b.x] = dev(1.0 / 9.0, -vy);
    dst[5 * N + b.rowm + b.xm] = dev(1.0 / 36.0, vx + vy);
    dst[6 * N + b.rowm + b.xp] = dev(1.0 / 36.0, -vx + vy);
    dst[7 * N + b.rowp + b.xp] = dev(1.0 / 36.0, -vx - vy);
    dst[8 * N + b.rowp + b.xm] = dev(1.0 / 36.0, vx - vy);
}

template <typename T>
__global__ void __launch_bounds__(256) k_moments(const T* src, const uint8_t* flags, double* rho, double* ux,
                                                 double* uy, uint32_t n, uint32_t nx, uint32_t ny, double rho0,
                                                 double ax, double ay)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    if (flags[s] == kSolid) {
        rho[s] = 0.0;
        ux[s] = 0.0;
        uy[s] = 0.0;
        return;
    }
    const Nbr b = neighbours(s, nx, ny);
    const Pop<T> p = pull(src, n, s, b);
    double dr, r, u, v;
    macro_fp64(p, rho0, ax, ay, dr, r, u, v);
    rho[s] = r;
    ux[s] = u;
    uy[s] = v;
}

constexpr int kRedBlock = 256;
constexpr uint32_t kRedMaxBlocks = 2048;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-level fixed-order sum of three values; result valid in thread 0.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c)
{
    __shared__ double sh[3][kRedBlock / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) {
        sh[0][w] = a;
        sh[1][w] = b;
        sh[2][w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = b = c = 0.0;
        for (int i = 0; i < kRedBlock / 64; ++i) {
            a += sh[0][i];
            b += sh[1][i];
            c += sh[2][i];
        }
    }
}

// Grid-stride partial sums: sum |u - u_prev|^2, sum |u|^2, sum (rho - rho0) over fluid sites.
template <typename T>
__global__ void __launch_bounds__(kRedBlock) k_residual_partial(const ReduceArgs a)
{
    const T* src = static_cast<const T*>(a.src);
    double s_du = 0.0, s_u = 0.0, s_dr = 0.0;
    const uint32_t stride = gridDim.x * kRedBlock;
    for (uint32_t s = blockIdx.x * kRedBlock + threadIdx.x; s < a.n; s += stride) {
        if (a.flags[s] == kSolid) continue;
        const Nbr b = neighbours(s, a.nx, a.ny);
        const Pop<T> p = pull(src, a.n, s, b);
        double dr, r, u, v;
        macro_fp64(p, a.rho0, a.ax, a.ay, dr, r, u, v);
        const double du = u - a.ux_prev[s], dv = v - a.uy_prev[s];
        s_du += du * du + dv * dv;
        s_u += u * u + v * v;
        s_dr += dr;
    }
    block_sum3(s_du, s_u, s_dr);
    if (threadIdx.x == 0) {
        a.partial[3 * blockIdx.x + 0] = s_du;
        a.partial[3 * blockIdx.x + 1] = s_u;
        a.partial[3 * blockIdx.x + 2] = s_dr;
    }
}

__global__ void __launch_bounds__(kRedBlock) k_residual_final(const double* partial, uint32_t nblocks, double* out)
{
    double x = 0.0, y = 0.0, z = 0.0;
    for (uint32_t i = threadIdx.x; i < nblocks; i += kRedBlock) {
        x += partial[3 * i + 0];
        y += partial[3 * i + 1];
        z += partial[3 * i + 2];
    }
    block_sum3(x, y, z);
    if (threadIdx.x == 0) {
        out[0] = x;
        out[1] = y;
        out[2] = z;
    }
}

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return static_cast<uint32_t>((a + b - 1) / b); }

template <typename T, int BLOCK>
hipError_t launch_step_block(const StepArgs<T>& a, bool write_u, bool node, hipStream_t stream)
{
    const uint32_t grid = ceil_div(a.n, BLOCK);
    if (write_u) {
        if (node)
            hipLaunchKernelGGL((k_step<T, true, true, BLOCK>), dim3(grid), dim3(BLOCK), 0, stream, a);
        else
            hipLaunchKernelGGL((k_step<T, true, false, BLOCK>), dim3(grid), dim3(BLOCK), 0, stream, a);
    } else {
        if (node)
            hipLaunchKernelGGL((k_step<T, false, true, BLOCK>), dim3(grid), dim3(BLOCK), 0, stream, a);
        else
            hipLaunchKernelGGL((k_step<T, false, false, BLOCK>), dim3(grid), dim3(BLOCK), 0, stream, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step_t(StepArgs<T> a, int block, bool write_u, bool node, hipStream_t stream)
{
    // the XCD remap covers the leading multiple of 8 blocks
    if (a.remap_blocks) a.remap_blocks = (ceil_div(a.n, block) / 8u) * 8u;
    switch (block) {
    case 64: return launch_step_block<T, 64>(a, write_u, node, stream);
    case 128: return launch_step_block<T, 128>(a, write_u, node, stream);
    case 512: return launch_step_block<T, 512>(a, write_u, node, stream);
    case 1024: return launch_step_block<T, 1024>(a, write_u, node, stream);
    default: return launch_step_block<T, 256>(a, write_u, node, stream);
    }
}

}  // namespace

hipError_t launch_step_f64(const StepArgs<double>& a, int block, bool write_u, bool node, hipStream_t stream)
{
    return launch_step_t<double>(a, block, write_u, node, stream);
}

hipError_t launch_step_f32(const StepArgs<float>& a, int block, bool write_u, bool node, hipStream_t stream)
{
    return launch_step_t<float>(a, block, write_u, node, stream);
}

hipError_t launch_precompute(const LinkInput& in, const PrecomputeArgs& a, double* coef64, float* coef32,
                             hipStream_t stream)
{
    if (a.n_links == 0) return hipSuccess;
    hipLaunchKernelGGL(k_precompute, dim3(ceil_div(a.n_links, 256)), dim3(256), 0, stream, in, a, coef64, coef32);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* ptr, uint64_t bytes, hipStream_t stream)
{
    if (bytes == 0) return hipSuccess;
    if ((reinterpret_cast<uintptr_t>(ptr) & 15u) == 0 && (bytes & 15u) == 0) {
        const uint64_t n16 = bytes / 16;
        hipLaunchKernelGGL(k_fill_zero, dim3(ceil_div(n16, 256)), dim3(256), 0, stream, static_cast<uint4*>(ptr),
                           n16);
    } else {
        hipLaunchKernelGGL(k_fill_zero_bytes, dim3(ceil_div(bytes, 256)), dim3(256), 0, stream,
                           static_cast<uint8_t*>(ptr), bytes);
    }
    return hipGetLastError();
}

hipError_t launch_init_fields(bool fp32, void* dst, const uint8_t* flags, const double* rho, const double* ux,
                              const double* uy, uint32_t n, uint32_t nx, uint32_t ny, double rho0, double ax,
                              double ay, hipStream_t stream)
{
    const dim3 grid(ceil_div(n, 256)), blk(256);
    if (fp32)
        hipLaunchKernelGGL(k_init_fields<float>, grid, blk, 0, stream, static_cast<float*>(dst), flags, rho, ux, uy,
                           n, nx, ny, rho0, ax, ay);
    else
        hipLaunchKernelGGL(k_init_fields<double>, grid, blk, 0, stream, static_cast<double*>(dst), flags, rho, ux,
                           uy, n, nx, ny, rho0, ax, ay);
    return hipGetLastError();
}

hipError_t launch_moments(bool fp32, const void* src, const uint8_t* flags, double* rho, double* ux, double* uy,
                          uint32_t n, uint32_t nx, uint32_t ny, double rho0, double ax, double ay,
                          hipStream_t stream)
{
    const dim3 grid(ceil_div(n, 256)), blk(256);
    if (fp32)
        hipLaunchKernelGGL(k_moments<float>, grid, blk, 0, stream, static_cast<const float*>(src), flags, rho, ux, uy,
                           n, nx, ny, rho0, ax, ay);
    else
        hipLaunchKernelGGL(k_moments<double>, grid, blk, 0, stream, static_cast<const double*>(src), flags, rho, ux,
                           uy, n, nx, ny, rho0, ax, ay);
    return hipGetLastError();
}

uint32_t residual_blocks(uint32_t n)
{
    const uint32_t b = ceil_div(n, kRedBlock);
    return b < kRedMaxBlocks ? (b == 0 ? 1u : b) : kRedMaxBlocks;
}

hipError_t launch_residual(bool fp32, const ReduceArgs& a, double* out, hipStream_t stream)
{
    const uint32_t nb = residual_blocks(a.n);
    if (fp32)
        hipLaunchKernelGGL(k_residual_partial<float>, dim3(nb), dim3(kRedBlock), 0, stream, a);
    else
        hipLaunchKernelGGL(k_residual_partial<double>, dim3(nb), dim3(kRedBlock), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(kRedBlock), 0, stream, a.partial, nb, out);
    return hipGetLastError();
}

}  // namespace lbm
