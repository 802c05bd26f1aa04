// HIP kernels of liblbm for gfx950 (CDNA4, 64-wide wavefronts).
//
// Storage: populations as deviations g_i = f_i - w_i rho0 from the rest equilibrium, in nine
// planes (structure of arrays) of n sites each, in "pull" layout: plane i at site y holds the
// value that site y + c_i receives at the next time level.  A fluid site reads its nine incoming
// populations at x - c_i (one coalesced, possibly one-element-shifted, load per plane) and writes
// its outgoing post-collision values at its own index (fully coalesced).
//
// Stores are issued for whole 128-byte lines: a line that is only partly written costs a
// read-modify-write in the memory system (measured: masking the stores of solid sites made a
// step 50% slower than streaming every site, while masking their loads cost nothing).  So every
// fluid site stores all nine planes (the value heading into a wall lands in a slot nobody reads),
// and a solid site stores zeros into its own, never-read slots whenever its line also holds a
// fluid site; lines that are entirely solid are skipped.
//
// Wall links: for a link (x, d) (x + c_d solid) the population i = opposite(d) that x receives at
// t + 1 is given by the boundary rule of Eq. (EqNewBDSC).  It is kept in a per-link array, indexed
// by the link's position in the (site, direction)-sorted link list, instead of in the solid
// neighbour's plane slot: the pull then selects, per lane, the plane or the link array (one load
// instruction per direction), and the boundary values are written link-parallel and coalesced.
//
// The boundary rule needs g_ibar(x, t), g'_i(x, t), g'_ibar(x, t), rho and the diffuse term, all
// in the registers of the thread that collides x.  The thread deposits them in LDS; after a
// barrier the block's threads walk the block's contiguous link range one link per thread, load
// the link coefficients (coalesced) and store the boundary value (coalesced).
//
// The single-step kernel is bound by HBM traffic (about 1-2 flop per byte).  The two-step kernel
// moves about half the bytes per step and is bound instead by the cache lines each CU can have in
// flight and by vector issue.  The 9x9 moment transform is applied in closed form with additions
// only, not as a dense contraction.
#include <hip/hip_runtime.h>

#include "lbm_internal.hpp"

namespace lbm {
namespace {

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

// Exclusive prefix over the wavefront of a per-lane count in [0, 15]; every lane must take part.
__device__ __forceinline__ uint32_t wave_prefix4(uint32_t v)
{
    const uint64_t b0 = __ballot(v & 1u);
    const uint64_t b1 = __ballot(v & 2u);
    const uint64_t b2 = __ballot(v & 4u);
    const uint64_t b3 = __ballot(v & 8u);
    return lanes_below(b0) + 2u * lanes_below(b1) + 4u * lanes_below(b2) + 8u * lanes_below(b3);
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// True when the 128-byte line holding this lane's element (elements of `bytes` bytes, lines
// aligned to the wavefront's first site) contains at least one lane with `any` set.  Every lane
// must take part.
__device__ __forceinline__ bool line_has(bool any, int bytes)
{
    const uint64_t m = __ballot(any);
    const int per = 128 / bytes;  // lanes per line: 32 (fp32) or 16 (fp64)
    const int lane = static_cast<int>(__lane_id());
    const uint64_t grp = (per >= 64) ? ~0ull : (((1ull << per) - 1ull) << (lane & ~(per - 1)));
    return (m & grp) != 0ull;
}

// Rank of link direction d (1..8) among the links of a site with flag byte fl.
__device__ __forceinline__ uint32_t rank_of(uint32_t fl, int d)
{
    return d == 1 ? 0u : static_cast<uint32_t>(__popc(__builtin_amdgcn_ubfe(fl, 0u, static_cast<uint32_t>(d - 1))));
}

// The flag byte as an opaque 32-bit value.  The compiler knows a byte load is below 256 and then
// tests single bits through sub-dword selects that cost an extra move each; hiding the range lets
// every test take one AND with an inline constant.  Applied only where the flags are tested after
// the loads that do not depend on them have been issued (the value must be present here).
__device__ __forceinline__ uint32_t opaque_flags(uint32_t fl)
{
    asm("" : "+v"(fl));
    return fl;
}

// Bit d - 1 of the flag byte: site has a wall link in direction d.
__device__ __forceinline__ bool has_link(uint32_t fl, int d)
{
    return __builtin_amdgcn_ubfe(fl, static_cast<uint32_t>(d - 1), 1u) != 0u;
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

// Flag byte of site s and the index of its first wall link.  Lanes past the end read as solid.
struct SiteLinks {
    uint32_t fl, k0;
};

__device__ __forceinline__ SiteLinks site_links(const Geo& g, uint32_t s)
{
    SiteLinks r;
    r.fl = (s < g.n) ? static_cast<uint32_t>(g.flags[s]) : kSolid;
    const uint32_t nlink = (r.fl != kSolid) ? static_cast<uint32_t>(__popc(r.fl)) : 0u;
    const uint32_t pre = wave_prefix4(nlink);
    // waves past the end read the final entry (index nchunks)
    r.k0 = static_cast<uint32_t>(g.chunk_base[uniform(min(s / kChunk, g.nchunks))]) + pre;
    return r;
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

// 1 / x: the correctly rounded quotient in fp64; in fp32 the hardware reciprocal (1 ulp) refined by
// one Newton step, which replaces the ten-instruction IEEE division sequence.
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Loads and stores at a wave-uniform base plus a 32-bit per-lane byte offset, which the hardware
// takes as a scalar base register plus one vector offset (no per-lane 64-bit address arithmetic).
template <typename T>
__device__ __forceinline__ T ld_at(const T* __restrict__ base, uint32_t off)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const unsigned char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ void st_at(T* __restrict__ base, uint32_t off, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(base) + off) = v;
}

// The nine incoming populations g_i(x, t) (D2Q9 order of Eq. (Eq3)).
template <typename T>
struct Pop {
    T g0, g1, g2, g3, g4, g5, g6, g7, g8;
};

// Population i of site s: from plane i at s - c_i, or from the link array when the upstream
// neighbour is a wall (link toward d = opposite(i)).  One load with a per-lane address.
#define LBM_PULL(I, D, UP)                                                                     \
    ((fl & (1u << ((D) - 1))) ? lnk[k0 + rank_of(fl, (D))] : pop[(I) * ps + (UP)])

template <typename T>
__device__ __forceinline__ Pop<T> pull(const T* __restrict__ pop, const T* __restrict__ lnk, uint64_t ps, uint32_t s,
                                       const Nbr& b, uint32_t fl, uint32_t k0)
{
    Pop<T> p;
    p.g0 = pop[s];
    p.g1 = LBM_PULL(1, 3, b.row + b.xm);   // from (x-1, y)
    p.g2 = LBM_PULL(2, 4, b.rowm + b.x);   // from (x, y-1)
    p.g3 = LBM_PULL(3, 1, b.row + b.xp);   // from (x+1, y)
    p.g4 = LBM_PULL(4, 2, b.rowp + b.x);   // from (x, y+1)
    p.g5 = LBM_PULL(5, 7, b.rowm + b.xm);  // from (x-1, y-1)
    p.g6 = LBM_PULL(6, 8, b.rowm + b.xp);  // from (x+1, y-1)
    p.g7 = LBM_PULL(7, 5, b.rowp + b.xp);  // from (x+1, y+1)
    p.g8 = LBM_PULL(8, 6, b.rowp + b.xm);  // from (x-1, y+1)
    return p;
}
#undef LBM_PULL

// The same nine values for a wavefront whose 64 sites lie in one lattice row: the rows y, y - 1 and
// y + 1 are wave-uniform, so each plane is read at a scalar row base plus the lane's byte offset of
// x, x - 1 or x + 1.  The loads do not depend on the site's flags (solid sites read slots they then
// ignore), so they are in flight together with the flag load.
template <typename T>
__device__ __forceinline__ Pop<T> pull_planes(const T* __restrict__ pop, uint64_t ps, uint64_t row, uint64_t rowm,
                                              uint64_t rowp, uint32_t x, uint32_t xm, uint32_t xp)
{
    const uint32_t ox = x * sizeof(T), om = xm * sizeof(T), op = xp * sizeof(T);
    Pop<T> p;
    p.g0 = ld_at(pop + row, ox);
    p.g1 = ld_at(pop + 1 * ps + row, om);   // from (x-1, y)
    p.g2 = ld_at(pop + 2 * ps + rowm, ox);  // from (x, y-1)
    p.g3 = ld_at(pop + 3 * ps + row, op);   // from (x+1, y)
    p.g4 = ld_at(pop + 4 * ps + rowp, ox);  // from (x, y+1)
    p.g5 = ld_at(pop + 5 * ps + rowm, om);  // from (x-1, y-1)
    p.g6 = ld_at(pop + 6 * ps + rowm, op);  // from (x+1, y-1)
    p.g7 = ld_at(pop + 7 * ps + rowp, op);  // from (x+1, y+1)
    p.g8 = ld_at(pop + 8 * ps + rowp, om);  // from (x-1, y+1)
    return p;
}

// Replaces the populations that come from a wall by the link array entries of a fluid site with flag
// byte fl (nonzero, not solid) whose first link is k0.
template <typename T>
__device__ __forceinline__ void pull_links(Pop<T>& p, const T* __restrict__ lnk, uint32_t fl, uint32_t k0)
{
    const uint32_t f = opaque_flags(fl);
    const T* __restrict__ lk = lnk + k0;
    if (has_link(f, 3)) p.g1 = lk[rank_of(f, 3)];
    if (has_link(f, 4)) p.g2 = lk[rank_of(f, 4)];
    if (has_link(f, 1)) p.g3 = lk[0];
    if (has_link(f, 2)) p.g4 = lk[rank_of(f, 2)];
    if (has_link(f, 7)) p.g5 = lk[rank_of(f, 7)];
    if (has_link(f, 8)) p.g6 = lk[rank_of(f, 8)];
    if (has_link(f, 5)) p.g7 = lk[rank_of(f, 5)];
    if (has_link(f, 6)) p.g8 = lk[rank_of(f, 6)];
}

// The wall populations of a wavefront whose 64 sites are one chunk, whose links are entries
// [kb, kb + n) of the link array in site order.  Lane i holds entry kb + i (i < 64), loaded along with
// the plane values (lv); a site whose first link is kb + rel0 then takes each of its entries from the
// owning lane with a cross-lane permute, done once per link direction that some site of the wave has.
// Entries past the first 64 of the chunk are loaded directly.
template <typename T>
__device__ __forceinline__ void pull_links_row(Pop<T>& p, T lv, const T* __restrict__ lnk, uint32_t fl, uint32_t rel0,
                                               uint32_t k0)
{
    const bool fluid = fl != kSolid;
    auto take = [&](int d, T& gv) __attribute__((always_inline)) {
        const bool mine = fluid && has_link(fl, d);
        if (__ballot(mine)) {
            const uint32_t rel = rel0 + rank_of(fl, d);
            const T v = __shfl(lv, static_cast<int>(rel & 63u));
            if (mine) gv = (rel < 64u) ? v : lnk[k0 + rank_of(fl, d)];
        }
    };
    take(3, p.g1);  // from (x-1, y)
    take(4, p.g2);  // from (x, y-1)
    take(1, p.g3);  // from (x+1, y)
    take(2, p.g4);  // from (x, y+1)
    take(7, p.g5);  // from (x-1, y-1)
    take(8, p.g6);  // from (x+1, y-1)
    take(5, p.g7);  // from (x+1, y+1)
    take(6, p.g8);  // from (x-1, y+1)
}

// The wall populations of a site whose chunk's first 64 link entries have been copied to LDS
// (stage[j] = entry kb + j); rel0 is the site's first link relative to kb.  Entries past the first
// 64 of the chunk are loaded directly.
template <typename T>
__device__ __forceinline__ void pull_links_staged(Pop<T>& p, const T* stage, const T* __restrict__ lnk, uint32_t fl,
                                                  uint32_t rel0, uint32_t k0)
{
    auto take = [&](int d, T& gv) __attribute__((always_inline)) {
        if (has_link(fl, d)) {
            const uint32_t rel = rel0 + rank_of(fl, d);
            gv = stage[rel & 63u];  // an LDS read in every case (a shared load would be a flat one)
            if (rel >= 64u) gv = lnk[k0 + rank_of(fl, d)];
        }
    };
    take(3, p.g1);  // from (x-1, y)
    take(4, p.g2);  // from (x, y-1)
    take(1, p.g3);  // from (x+1, y)
    take(2, p.g4);  // from (x, y+1)
    take(7, p.g5);  // from (x-1, y-1)
    take(8, p.g6);  // from (x+1, y-1)
    take(5, p.g7);  // from (x+1, y+1)
    take(6, p.g8);  // from (x-1, y+1)
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

// Result of one collision: the post-collision deviations h_i = g'_i and the macroscopic values
// the boundary rule needs.
template <typename T>
struct Post {
    T h0, h1, h2, h3, h4, h5, h6, h7, h8;
    T dr, rho, ux, uy, u2;
};

// Collision of one fluid site in moment space (Eqs. (LBEColli), (LBEforce), (MomentPost)) on the
// deviations g_i = f_i - w_i rho0; shared by every step kernel so that they agree bit for bit.
template <typename T>
__device__ __forceinline__ void collide(const Pop<T>& p, const StepArgs<T>& a, Post<T>& o)
{
    const T g0 = p.g0, g1 = p.g1, g2 = p.g2, g3 = p.g3, g4 = p.g4, g5 = p.g5, g6 = p.g6, g7 = p.g7, g8 = p.g8;
    // conserved moments and half-force velocity, Eq. (FluidMacr)
    const T s14 = (g1 + g2) + (g3 + g4);
    const T s58 = (g5 + g6) + (g7 + g8);
    const T dr = g0 + s14 + s58;
    const T rho = a.rho0 + dr;
    const T jx = (g1 - g3) + (g5 - g6) + (g8 - g7);
    const T jy = (g2 - g4) + (g5 + g6) - (g7 + g8);
    const T irho = recip(rho);
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
    const T pxxp =
        pxx - a.s_s * (pxx - rho * (ux * ux - uy * uy)) + a.c_s * (T(2) * rho * (ux * a.ax - uy * a.ay));
    const T pxyp = pxy - a.s_s * (pxy - rho * (ux * uy)) + a.c_s * (rho * (ux * a.ay + uy * a.ax));
    // conserved: rho' = rho; j' = j + rho a exactly (the tau_j relaxation and forcing cancel)
    const T jxp = jx + rho * a.ax;
    const T jyp = jy + rho * a.ay;

    // f' = M^-1 m' with M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
    // The conserved moments (rho, j) never relax, so a rounded constant 1/9 or 1/6 would scale
    // mass and momentum by (1 + its rounding error) at every collision and the bias would grow
    // over the whole run; they are divided with a two-term constant (error below one ulp,
    // unbiased).
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

    o.h0 = h0;
    o.h1 = h1;
    o.h2 = h2;
    o.h3 = h3;
    o.h4 = h4;
    o.h5 = h5;
    o.h6 = h6;
    o.h7 = h7;
    o.h8 = h8;
    o.dr = dr;
    o.rho = rho;
    o.ux = ux;
    o.uy = uy;
    o.u2 = u2;
}

// Boundary value of Eq. (EqNewBDSC) in deviation form for link k:
//   g_i(x, t+1) = a1 g_ibar + a2 g'_i + a3 g'_ibar + beta rho + kappa w_i (drho + rho phi_i(u)).
template <typename T>
struct LinkCoefs {
    T a1, a2, a3, beta, kappa;
};
template <typename T>
__device__ __forceinline__ LinkCoefs<T> link_coefs(const LinkCoef<T>& c, uint32_t k)
{
    return LinkCoefs<T>{c.a1[k], c.a2[k], c.a3[k], c.beta[k], c.kappa[k]};
}
template <typename T>
__device__ __forceinline__ T link_value(const LinkCoefs<T>& w, T gb, T hi, T hb, T rho, T wdif)
{
    return w.a1 * gb + w.a2 * hi + w.a3 * hb + w.beta * rho + w.kappa * wdif;
}
template <typename T>
__device__ __forceinline__ T link_value(const LinkCoef<T>& c, uint32_t k, T gb, T hi, T hb, T rho, T wdif)
{
    return link_value(link_coefs(c, k), gb, hi, hb, rho, wdif);
}

// w_i (drho + rho phi_i(u)) (node reading) or w_i drho (wall reading, where the wall equilibrium
// is folded into beta), phi_i(u) = 3 c_i.u + 4.5 (c_i.u)^2 - 1.5 u^2 with cu = c_i.u.
// With the site parts b = drho - 1.5 rho u^2 (node reading; b = drho in the wall reading), 3 rho and
// 4.5 rho formed once per site, the term of link direction i is w_i (b + c_i.u (3 rho + 4.5 rho c_i.u)).
template <typename T>
struct DiffuseSite {
    T b, r3, r45;
};
template <typename T, bool NODE>
__device__ __forceinline__ DiffuseSite<T> diffuse_base(T dr, T rho, T u2)
{
    return DiffuseSite<T>{NODE ? dr - T(1.5) * rho * u2 : dr, T(3) * rho, T(4.5) * rho};
}
template <typename T, bool NODE>
__device__ __forceinline__ T diffuse_term(T w, const DiffuseSite<T>& ds, T cu)
{
    return NODE ? w * (cu * (ds.r45 * cu + ds.r3) + ds.b) : w * ds.b;
}

// Calls fn(d, rank, g_ibar, g'_i, g'_ibar, w_i, c_i.u) for every wall link direction d of a site
// with flag byte fl (the unknown population is i = opposite(d); rank = the link's position among
// the site's links).
template <typename T, typename F>
__device__ __forceinline__ void for_links(uint32_t fl, const Pop<T>& p, const Post<T>& o, F&& fn)
{
    const T w1 = T(1.0 / 9.0), w5 = T(1.0 / 36.0);
    if (has_link(fl, 1)) fn(1, 0u, p.g1, o.h3, o.h1, w1, -o.ux);                  // toward E, unknown W
    if (has_link(fl, 2)) fn(2, rank_of(fl, 2), p.g2, o.h4, o.h2, w1, -o.uy);      // toward N, unknown S
    if (has_link(fl, 3)) fn(3, rank_of(fl, 3), p.g3, o.h1, o.h3, w1, o.ux);       // toward W, unknown E
    if (has_link(fl, 4)) fn(4, rank_of(fl, 4), p.g4, o.h2, o.h4, w1, o.uy);       // toward S, unknown N
    if (has_link(fl, 5)) fn(5, rank_of(fl, 5), p.g5, o.h7, o.h5, w5, -o.ux - o.uy);  // toward NE, unknown SW
    if (has_link(fl, 6)) fn(6, rank_of(fl, 6), p.g6, o.h8, o.h6, w5, o.ux - o.uy);   // toward NW, unknown SE
    if (has_link(fl, 7)) fn(7, rank_of(fl, 7), p.g7, o.h5, o.h7, w5, o.ux + o.uy);   // toward SW, unknown NE
    if (has_link(fl, 8)) fn(8, rank_of(fl, 8), p.g8, o.h6, o.h8, w5, -o.ux + o.uy);  // toward SE, unknown NW
}

// LDS staging of one link's operands, one record per link (the five stores of a link share one
// address).
template <typename T>
struct LinkRec {
    T gb;   // g_ibar(x, t), pre-collision, toward the wall
    T hi;   // g'_i(x, t), post-collision, away from the wall
    T hb;   // g'_ibar(x, t)
    T rho;  // rho(x, t)
    T dif;  // w_i (drho + rho phi_i(u)) in the node reading, w_i drho in the wall reading
};

template <typename T>
__device__ __forceinline__ T link_value(const LinkCoef<T>& c, uint32_t k, const LinkRec<T>& r)
{
    return link_value(c, k, r.gb, r.hi, r.hb, r.rho, r.dif);
}
template <typename T>
__device__ __forceinline__ T link_value(const LinkCoefs<T>& w, const LinkRec<T>& r)
{
    return link_value(w, r.gb, r.hi, r.hb, r.rho, r.dif);
}

// One tile of BLOCK consecutive sites starting at `start` (a multiple of BLOCK) of the lattice
// described by a.g: collision and streaming of its fluid sites, then the boundary values of its
// wall links.  Shared by the single-lattice kernel and the batched persistent kernel, so that both
// compute bit-identical results.
template <typename T, bool WRITE_U, bool NODE, int BLOCK>
__device__ __forceinline__ void step_tile(const StepArgs<T>& a, uint32_t start, unsigned char* lds_raw)
{
    const Geo& g = a.g;
    const uint32_t s = start + threadIdx.x;
    // link range of this tile (uniform, scalar loads)
    const uint32_t c0 = start / kChunk;
    const uint32_t c1 = min(c0 + BLOCK / kChunk, g.nchunks);
    const uint32_t kblk = static_cast<uint32_t>(g.chunk_base[c0]);
    const uint32_t nl_blk = static_cast<uint32_t>(g.chunk_base[c1]) - kblk;
    const SiteLinks sl = site_links(g, s);
    const uint32_t fl = sl.fl, k0 = sl.k0;
    const uint64_t ps = g.ps;
    const bool store_line = line_has(fl != kSolid, sizeof(T));

    LinkRec<T>* st = reinterpret_cast<LinkRec<T>*>(lds_raw);

    if (fl != kSolid) {
        const Nbr b = neighbours(s, g.nx, g.ny);
        const Pop<T> p = pull(a.src.pop, a.src.link, ps, s, b, fl, k0);
        if (WRITE_U) {
            double dr_d, rho_d, ux_d, uy_d;
            macro_fp64(p, static_cast<double>(a.rho0), static_cast<double>(a.ax), static_cast<double>(a.ay),
                       dr_d, rho_d, ux_d, uy_d);
            a.ux_out[s] = ux_d;
            a.uy_out[s] = uy_d;
        }

        Post<T> o;
        collide(p, a, o);
        const T dr = o.dr, rho = o.rho, u2 = o.u2;
        const T h0 = o.h0, h1 = o.h1, h2 = o.h2, h3 = o.h3, h4 = o.h4, h5 = o.h5, h6 = o.h6, h7 = o.h7, h8 = o.h8;

        // Post-collision values leave along c_i and are pulled by x + c_i (the ones heading into
        // a wall are stored too, into slots nobody reads, to keep the lines whole).
        T* __restrict__ dst = a.dst.pop;
        dst[s] = h0;
        dst[1 * ps + s] = h1;
        dst[2 * ps + s] = h2;
        dst[3 * ps + s] = h3;
        dst[4 * ps + s] = h4;
        dst[5 * ps + s] = h5;
        dst[6 * ps + s] = h6;
        dst[7 * ps + s] = h7;
        dst[8 * ps + s] = h8;

        if (fl) {
            // operands of Eq. (EqNewBDSC) for each wall link (x, d); the unknown is i = opposite(d)
            LinkRec<T>* sp = st + (k0 - kblk);
            const DiffuseSite<T> b = diffuse_base<T, NODE>(dr, rho, u2);
            for_links(fl, p, o, [&](int, uint32_t rank, T gb, T hi, T hb, T w, T cu) {
                sp[rank] = LinkRec<T>{gb, hi, hb, rho, diffuse_term<T, NODE>(w, b, cu)};
            });
        }
    }
    // solid sites that share a line with a fluid site: zeros in never-read slots keep the stores
    // whole lines (a separate branch after the fluid one, so that a mixed wave issues its loads first)
    if (fl == kSolid && store_line && s < g.n) {
        T* __restrict__ dst = a.dst.pop;
#pragma unroll
        for (int i = 0; i < 9; ++i) dst[i * ps + s] = T(0);
    }

    if (nl_blk != 0) {  // block-uniform
        __syncthreads();
        // link-parallel phase: Eq. (EqNewBDSC) in deviation form,
        //   g_i(x, t+1) = a1 g_ibar + a2 g'_i + a3 g'_ibar + beta rho + kappa w_i (drho + rho phi_i(u))
        const LinkCoef<T> c = a.coef;
        for (uint32_t j = threadIdx.x; j < nl_blk; j += BLOCK) {
            const uint32_t k = kblk + j;
            a.dst.link[k] = link_value(c, k, st[j]);
        }
    }
}

template <typename T, bool WRITE_U, bool NODE, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_step(const StepArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    step_tile<T, WRITE_U, NODE, BLOCK>(a, blockIdx.x * BLOCK, lds_raw);
}

// ------------------------------------------------------- two time steps per launch (fused)
//
// Temporal blocking: a block owns a tile of 64 x TY sites (64 = one chunk).  Step 1 runs on the
// tile and a one-site halo around it, RPW rows per wave and one more wave for the two halo columns:
// its sites pull from the global planes and link array of time t, collide, and leave their nine
// post-collision values in LDS; the tile's sites also stage the operands of their wall links, and
// after a barrier one link-parallel pass leaves each boundary value in the LDS slot of the solid
// neighbour x + c_d, which is exactly where step 2 pulls it.  Step 2 runs on the tile only, pulling
// from LDS, and stores time t + 2 to the global planes (whole lines) and its boundary values to the
// link array (link-parallel over the tile rows' contiguous link ranges, as in step_tile).  Each
// site's arithmetic is that of step_tile (same collide / link_value / diffuse_term), so two fused
// steps give the bits of two single steps.  Needs nx % 64 == 0 and ny % TY == 0.

// Step 1 of one site whose nine incoming populations p have been pulled: collision, the nine
// post-collision values into LDS row rr, column cc, and (tile sites only) the operands of each of
// its wall links into the staging area at j0 + rank, with the LDS slot of the solid neighbour
// x + c_d that will receive the boundary value.
template <typename T, bool NODE>
__device__ __forceinline__ void fused_finish1(const StepArgs<T>& a, T* F, LinkRec<T>* st, uint32_t* tg,
                                              const Pop<T>& p, uint32_t fl, uint32_t j0, int rr, int cc,
                                              bool in_tile, int W, int P)
{
    Post<T> o;
    collide(p, a, o);
    const int idx = rr * W + cc;
    F[idx] = o.h0;
    F[1 * P + idx] = o.h1;
    F[2 * P + idx] = o.h2;
    F[3 * P + idx] = o.h3;
    F[4 * P + idx] = o.h4;
    F[5 * P + idx] = o.h5;
    F[6 * P + idx] = o.h6;
    F[7 * P + idx] = o.h7;
    F[8 * P + idx] = o.h8;
    if (in_tile && fl) {
        LinkRec<T>* sp = st + j0;
        uint32_t* tp = tg + j0;
        const DiffuseSite<T> b = diffuse_base<T, NODE>(o.dr, o.rho, o.u2);
        for_links(fl, p, o, [&](int d, uint32_t j, T gb, T hi, T hb, T w, T cu) {
            // c_d and the unknown direction i = opposite(d)
            const int cx = (d == 1 || d == 5 || d == 8) ? 1 : ((d == 3 || d == 6 || d == 7) ? -1 : 0);
            const int cy = (d == 2 || d == 5 || d == 6) ? 1 : ((d == 4 || d == 7 || d == 8) ? -1 : 0);
            const int i = (d <= 4) ? ((d + 1) & 3) + 1 : ((d - 3) & 3) + 5;
            sp[j] = LinkRec<T>{gb, hi, hb, o.rho, diffuse_term<T, NODE>(w, b, cu)};
            tp[j] = static_cast<uint32_t>(i * P + (rr + cy) * W + (cc + cx));
        });
    }
}

// Tile of block b: blocks are dealt round-robin to the eight XCDs (b % 8), so block b is mapped to
// tile (b % 8) * (ntiles / 8) + b / 8; each XCD then walks its own contiguous run of tiles in
// row-major order and neighbouring tiles, whose halos overlap, meet in the same L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t ntiles)
{
    if (ntiles % 8u != 0u) return b;
    return (b % 8u) * (ntiles / 8u) + b / 8u;
}

// fp32 two-step tiles: block b still goes to XCD b % 8, but within the XCD block v = b / 8 walks
// bands of 4 tile rows x 32 tile columns, column-major within a band, so that v + 32 is the tile
// below v.  An XCD hands out its blocks to its 32 CUs in turn, so the tiles one CU holds at a time
// are stacked vertically and read each other's halo rows from that CU's L1 (measured: 2% over row
// order in fp32; 4-row bands beat 2-, 8- and 16-row ones; 16-column groups gain nothing; fp64 blocks,
// fewer and larger, lose with it).  Other tile counts keep xcd_tile.
__device__ __forceinline__ uint32_t band_tile(uint32_t b, uint32_t ntiles, uint32_t tiles_x)
{
    const uint32_t per = ntiles / 8u;
    if (ntiles % 8u != 0u || tiles_x % 32u != 0u || per % (4u * tiles_x) != 0u) return xcd_tile(b, ntiles);
    const uint32_t xg = b % 8u, v = b / 8u;
    const uint32_t band = v / (4u * tiles_x), w = v % (4u * tiles_x);
    const uint32_t grp = w / 128u, rem = w % 128u;
    return xg * per + (band * 4u + rem / 32u) * tiles_x + grp * 32u + rem % 32u;
}

// Block of the two-step kernel: (TY + 2) / RPW step-1 waves, each taking RPW LDS rows, and one wave
// for the two halo columns.
template <int TY, int RPW>
constexpr int step2_threads()
{
    return 64 * ((TY + 2) / RPW + 1);
}
template <typename T, bool WRITE_U, bool NODE, int TY, int RPW>
__global__ void __launch_bounds__((step2_threads<TY, RPW>())) k_step2(const StepArgs<T> a)
{
    static_assert((TY + 2) % RPW == 0 && TY % RPW == 0, "rows per wave must divide the tile rows");
    constexpr int W = kFuseTX + 2, R = TY + 2, P = R * W, NT = step2_threads<TY, RPW>();
    constexpr int NW1 = R / RPW;  // step-1 row waves; wave NW1 takes the halo columns
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* F = reinterpret_cast<T*>(lds_raw);  // [9][R][W] post-collision values of step 1
    LinkRec<T>* st = reinterpret_cast<LinkRec<T>*>(F + 9 * P);  // [lds_links] link operands (step 1, then 2)
    uint32_t* tg = reinterpret_cast<uint32_t*>(st + a.lds_links);     // [lds_links] F slot of each link
    uint32_t* j0s = tg + a.lds_links;                                     // [TY][64] first staging slot
    uint8_t* fls = reinterpret_cast<uint8_t*>(j0s + TY * kFuseTX);        // [TY][64] flag bytes

    const Geo& g = a.g;
    const uint32_t tiles_x = g.nx / kFuseTX;
    const uint32_t tile =
        sizeof(T) == 4 ? band_tile(blockIdx.x, gridDim.x, tiles_x) : xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t x0 = (tile % tiles_x) * kFuseTX, y0 = (tile / tiles_x) * TY;
    const int tid = threadIdx.x, lane = tid % 64;
    const int wave = static_cast<int>(uniform(static_cast<uint32_t>(tid) / 64u));
    const uint64_t ps = g.ps;

    // Link ranges of the tile rows (wave-uniform): row q owns links [kq[q], kq[q] + oq[q+1] - oq[q]),
    // staged from slot oq[q].
    uint32_t kq[TY], oq[TY + 1];
    oq[0] = 0;
#pragma unroll
    for (int q = 0; q < TY; ++q) {
        const uint32_t c = ((y0 + q) * g.nx + x0) / kChunk;
        kq[q] = static_cast<uint32_t>(g.chunk_base[c]);
        oq[q + 1] = oq[q] + (static_cast<uint32_t>(g.chunk_base[c + 1]) - kq[q]);
    }
    const uint32_t total = oq[TY];
    // link index of staging slot j
    auto link_of = [&](uint32_t j) __attribute__((always_inline)) {
        uint32_t k = j + kq[0];
#pragma unroll
        for (int q = 1; q < TY; ++q)
            if (j >= oq[q]) k = j - oq[q] + kq[q];
        return k;
    };
    // fp32: the coefficients of this thread's first staging slot are fetched now and used by both
    // steps (in fp64 the ten extra live registers would cost a resident block)
    const LinkCoef<T> c = a.coef;
    const bool has1 = sizeof(T) == 4 && static_cast<uint32_t>(tid) < total;
    const uint32_t k1 = link_of(static_cast<uint32_t>(tid));
    LinkCoefs<T> w1{};
    if (has1) w1 = link_coefs(c, k1);

    if (wave < NW1) {
        // step 1: wave w takes LDS rows w RPW .. w RPW + RPW - 1 (LDS row rr is tile row rr - 1;
        // rows -1 and TY are the halo rows).  Each row of a wave is one chunk of one lattice row,
        // so rows and chunks are wave-uniform.  With several rows per wave all are pulled before
        // any is collided; with one, pull and collision stay together (fewer live registers).
        uint32_t fl[RPW], k0[RPW], j0[RPW], kb[RPW], nrow[RPW], yr[RPW];
        Pop<T> p[RPW];
        T lv[RPW];
        // the rows' chunk offsets come first: scalar loads, all issued before any direct LDS load
        // (after one, the compiler no longer takes the offset table as unchanged)
#pragma unroll
        for (int h = 0; h < RPW; ++h) {
            const int rr = wave * RPW + h;
            yr[h] = (rr == 0) ? (y0 == 0 ? g.ny - 1 : y0 - 1) : ((y0 + rr - 1 == g.ny) ? 0 : y0 + rr - 1);
            const uint32_t c = static_cast<uint32_t>((uint64_t(yr[h]) * g.nx + x0) / kChunk);
            kb[h] = static_cast<uint32_t>(g.chunk_base[c]);
            nrow[h] = static_cast<uint32_t>(g.chunk_base[c + 1]) - kb[h];
        }
#pragma unroll
        for (int h = 0; h < RPW; ++h) {
            const int rr = wave * RPW + h;
            const uint32_t y = yr[h];
            const uint32_t ym = (y == 0) ? g.ny - 1 : y - 1, yp = (y + 1 == g.ny) ? 0 : y + 1;
            const uint64_t row = uint64_t(y) * g.nx;
            const uint32_t x = x0 + lane;
            const uint32_t xm = (x == 0) ? g.nx - 1 : x - 1, xp = (x + 1 == g.nx) ? 0 : x + 1;
            fl[h] = ld_at(g.flags + row, x);
            p[h] = pull_planes(a.src.pop, ps, row, uint64_t(ym) * g.nx, uint64_t(yp) * g.nx, x, xm, xp);
            // the row's first 64 link entries are fetched with the planes: in fp64 (one row per
            // wave) into a register of each lane; in fp32 straight into LDS, into this row's slots
            // of plane 0, which only this wave writes and only after it has read them
            if constexpr (RPW == 1) {
                lv[h] = (static_cast<uint32_t>(lane) < nrow[h]) ? a.src.link[kb[h] + lane] : T(0);
            } else {
                static_assert(sizeof(T) == 4, "direct LDS staging of link entries moves one dword per lane");
                if (static_cast<uint32_t>(lane) < nrow[h])
                    __builtin_amdgcn_global_load_lds(a.src.link + kb[h] + lane,
                                                     (__attribute__((address_space(3))) void*)(F + rr * W + 1), 4, 0, 0);
            }
        }
        if constexpr (RPW > 1) {
            // the compiler does not track the LDS writes of the direct loads: wait for them here
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        }
#pragma unroll
        for (int h = 0; h < RPW; ++h) {
            const int rr = wave * RPW + h;
            const uint32_t nlink = (fl[h] != kSolid) ? static_cast<uint32_t>(__popc(fl[h])) : 0u;
            k0[h] = kb[h] + wave_prefix4(nlink);
            j0[h] = 0;
            if (rr >= 1 && rr <= TY) {
                uint32_t off = 0;  // staging offset of this tile row: the links of the tile rows above
                if constexpr (RPW == 1) {
                    for (int q = 0; q < rr - 1; ++q) {
                        const uint32_t cq = ((y0 + q) * g.nx + x0) / kChunk;
                        off += static_cast<uint32_t>(g.chunk_base[cq + 1] - g.chunk_base[cq]);
                    }
                } else {
#pragma unroll
                    for (int q = 1; q < TY; ++q)
                        if (rr - 1 == q) off = oq[q];
                }
                j0[h] = off + (k0[h] - kb[h]);
                j0s[(rr - 1) * kFuseTX + lane] = j0[h];
                fls[(rr - 1) * kFuseTX + lane] = static_cast<uint8_t>(fl[h]);
            }
            if constexpr (RPW == 1)
                pull_links_row(p[h], lv[h], a.src.link, fl[h], k0[h] - kb[h], k0[h]);
            else if (fl[h] != kSolid && fl[h] != 0u)
                pull_links_staged(p[h], F + rr * W + 1, a.src.link, fl[h], k0[h] - kb[h], k0[h]);
            if constexpr (RPW == 1)
                if (fl[h] != kSolid)
                    fused_finish1<T, NODE>(a, F, st, tg, p[h], fl[h], j0[h], rr, lane + 1, rr >= 1 && rr <= TY, W, P);
        }
        if constexpr (RPW > 1) {
#pragma unroll
            for (int h = 0; h < RPW; ++h) {
                const int rr = wave * RPW + h;
                if (fl[h] != kSolid)
                    fused_finish1<T, NODE>(a, F, st, tg, p[h], fl[h], j0[h], rr, lane + 1, rr >= 1 && rr <= TY, W,
                                           P);
            }
        }
    } else if (lane < 2 * R) {
        // the last wave: halo columns x0 - 1 (last site of its chunk) and x0 + 64 (first of its
        // chunk)
        const int rr = lane >> 1, side = lane & 1;
        const uint32_t y = (rr == 0) ? (y0 == 0 ? g.ny - 1 : y0 - 1) : ((y0 + rr - 1 == g.ny) ? 0 : y0 + rr - 1);
        const uint32_t x = side ? ((x0 + kFuseTX == g.nx) ? 0 : x0 + kFuseTX) : (x0 == 0 ? g.nx - 1 : x0 - 1);
        const uint32_t s = y * g.nx + x;
        const uint32_t xm = (x == 0) ? g.nx - 1 : x - 1, xp = (x + 1 == g.nx) ? 0 : x + 1;
        const uint32_t ym = (y == 0) ? g.ny - 1 : y - 1, yp = (y + 1 == g.ny) ? 0 : y + 1;
        const uint32_t fl = g.flags[s];
        if (fl != kSolid) {
            const uint32_t cb = static_cast<uint32_t>(g.chunk_base[s / kChunk + (side ? 0u : 1u)]);
            const uint32_t k0 = side ? cb : cb - static_cast<uint32_t>(__popc(fl));
            Pop<T> p;
            if constexpr (sizeof(T) == 4) {
                // the nine plane values are requested before the link entries, which wait for the
                // chunk offset (measured faster in fp32)
                p = pull_planes(a.src.pop, ps, uint64_t(y) * g.nx, uint64_t(ym) * g.nx, uint64_t(yp) * g.nx, x, xm, xp);
                if (fl != 0u) pull_links(p, a.src.link, fl, k0);
            } else {
                // one load per population, from the plane or the link array
                Nbr b;
                b.x = x;
                b.xm = xm;
                b.xp = xp;
                b.row = y * g.nx;
                b.rowm = ym * g.nx;
                b.rowp = yp * g.nx;
                p = pull(a.src.pop, a.src.link, ps, s, b, fl, k0);
            }
            fused_finish1<T, NODE>(a, F, st, tg, p, fl, 0, rr, side ? W - 1 : 0, false, W, P);
        }
    }
    __syncthreads();

    // the boundary values of step 1, link-parallel, into the LDS slots of the solid neighbours
    if (has1) F[tg[tid]] = link_value(w1, st[tid]);
    for (uint32_t jj = has1 ? tid + NT : tid; jj < total; jj += NT)
        F[tg[jj]] = link_value(c, link_of(jj), st[jj]);
    __syncthreads();

    // step 2: pulling from LDS (with several rows per wave, all rows' LDS loads are issued first)
    auto load2 = [&](int r, Pop<T>& p) __attribute__((always_inline)) {
        const int idx = (r + 1) * W + lane + 1;
        p.g0 = F[idx];
        p.g1 = F[1 * P + idx - 1];      // from (x-1, y)
        p.g2 = F[2 * P + idx - W];      // from (x, y-1)
        p.g3 = F[3 * P + idx + 1];      // from (x+1, y)
        p.g4 = F[4 * P + idx + W];      // from (x, y+1)
        p.g5 = F[5 * P + idx - W - 1];  // from (x-1, y-1)
        p.g6 = F[6 * P + idx - W + 1];  // from (x+1, y-1)
        p.g7 = F[7 * P + idx + W + 1];  // from (x+1, y+1)
        p.g8 = F[8 * P + idx + W - 1];  // from (x-1, y+1)
    };
    auto finish2 = [&](int r, uint32_t fl, const Pop<T>& p) __attribute__((always_inline)) {
        const uint64_t row = uint64_t(y0 + r) * g.nx;
        const uint32_t s = static_cast<uint32_t>(row) + x0 + lane;
        const uint32_t ox = (x0 + lane) * sizeof(T);
        const bool store_line = line_has(fl != kSolid, sizeof(T));
        T* __restrict__ dst = a.dst.pop + row;
        if (fl != kSolid) {
            if (WRITE_U) {
                double dr_d, rho_d, ux_d, uy_d;
                macro_fp64(p, static_cast<double>(a.rho0), static_cast<double>(a.ax), static_cast<double>(a.ay),
                           dr_d, rho_d, ux_d, uy_d);
                a.ux_out[s] = ux_d;
                a.uy_out[s] = uy_d;
            }
            Post<T> o;
            collide(p, a, o);
            st_at(dst, ox, o.h0);
            st_at(dst + 1 * ps, ox, o.h1);
            st_at(dst + 2 * ps, ox, o.h2);
            st_at(dst + 3 * ps, ox, o.h3);
            st_at(dst + 4 * ps, ox, o.h4);
            st_at(dst + 5 * ps, ox, o.h5);
            st_at(dst + 6 * ps, ox, o.h6);
            st_at(dst + 7 * ps, ox, o.h7);
            st_at(dst + 8 * ps, ox, o.h8);
            if (fl) {
                LinkRec<T>* sp = st + j0s[r * kFuseTX + lane];
                const DiffuseSite<T> b = diffuse_base<T, NODE>(o.dr, o.rho, o.u2);
                for_links(fl, p, o, [&](int, uint32_t rank, T gb, T hi, T hb, T w, T cu) {
                    sp[rank] = LinkRec<T>{gb, hi, hb, o.rho, diffuse_term<T, NODE>(w, b, cu)};
                });
            }
        }
        if (fl == kSolid && store_line) {
#pragma unroll
            for (int i = 0; i < 9; ++i) st_at(dst + i * ps, ox, T(0));
        }
    };
    // one tile row per wave when the block has a wave for every row, else RPW rows per wave
    constexpr int RPW2 = (TY <= NW1 + 1) ? 1 : RPW;
    if (wave < TY / RPW2) {
        if constexpr (RPW2 == 1) {
            const uint32_t fl = fls[wave * kFuseTX + lane];
            Pop<T> p;
            if (fl != kSolid) load2(wave, p);
            finish2(wave, fl, p);
        } else {
            uint32_t fl[RPW2];
            Pop<T> p[RPW2];
#pragma unroll
            for (int h = 0; h < RPW2; ++h) {
                fl[h] = fls[(wave * RPW2 + h) * kFuseTX + lane];
                if (fl[h] != kSolid) load2(wave * RPW2 + h, p[h]);
            }
#pragma unroll
            for (int h = 0; h < RPW2; ++h) finish2(wave * RPW2 + h, fl[h], p[h]);
        }
    }
    __syncthreads();
    // the tile's boundary values of step 2, link-parallel over its rows' contiguous link ranges
    if (has1) a.dst.link[k1] = link_value(w1, st[tid]);
    for (uint32_t jj = has1 ? tid + NT : tid; jj < total; jj += NT) {
        const uint32_t k = link_of(jj);
        a.dst.link[k] = link_value(c, k, st[jj]);
    }
}

// View of instance `in` of a batch: its flags, chunk offsets and u record start at its site offset
// in the batch's site space; its planes are the batch planes shifted by the offset (same stride);
// link indices in the chunk table are global.
template <typename T>
__device__ __forceinline__ StepArgs<T> instance_args(const BatchArgs<T>& b, const BatchInst<T>& in)
{
    StepArgs<T> a;
    a.g = Geo{b.flags + in.off, b.chunk_base + in.off / kChunk, in.n, in.nx, in.ny, (in.n + kChunk - 1) / kChunk,
              b.ps};
    a.src = Level<T>{b.src.pop + in.off, b.src.link};
    a.dst = Level<T>{b.dst.pop + in.off, b.dst.link};
    a.coef = b.coef;
    a.ux_out = b.ux_out + in.off;
    a.uy_out = b.uy_out + in.off;
    a.lds_links = b.lds_links;
    a.rho0 = in.ph.rho0;
    a.ax = in.ph.ax;
    a.ay = in.ph.ay;
    a.s_e = in.ph.s_e;
    a.s_eps = in.ph.s_eps;
    a.s_q = in.ph.s_q;
    a.s_s = in.ph.s_s;
    a.c_e = in.ph.c_e;
    a.c_eps = in.ph.c_eps;
    a.c_q = in.ph.c_q;
    a.c_s = in.ph.c_s;
    return a;
}

// Persistent batched step: a fixed grid strides over the device-resident list of active tiles
// (instance, local start); retiring an instance only shrinks that list, so a captured graph of
// these launches stays valid.
template <typename T, bool WRITE_U, bool NODE, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_step_batch(const BatchArgs<T> b)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint32_t ntile = *b.n_active;
    for (uint32_t t = blockIdx.x; t < ntile; t += gridDim.x) {
        const TileRef tr = b.tiles[t];
        const StepArgs<T> a = instance_args(b, b.inst[tr.inst]);
        step_tile<T, WRITE_U, NODE, BLOCK>(a, tr.start, lds_raw);
        __syncthreads();  // the next tile reuses the LDS staging area
    }
}

// ------------------------------------------------------------------- per-link precompute

__device__ __forceinline__ double weight_of(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }

// Coefficients of Eq. (EqNewBDSC) per link from gamma, the l and r rules of Sec. III.B (or their
// counterparts under the wall reading) and the wall velocity; one thread per link, fp64.  Output rows of coef64 (n_links each):
// l_raw, l_eff, r, alpha1, alpha2, alpha3, beta, kappa.
__global__ void __launch_bounds__(256) k_precompute(const LinkInput in, const PrecomputeArgs a, double* coef64,
                                                    float* coef32)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= a.n_links) return;
    const int64_t nl = a.row_stride;
    const double g = in.q[k];
    const double ts = a.tau_s, L1 = a.L1, E = a.E, sq = a.sq6pi;
    const double t2 = 2.0 * ts - 1.0;
    // Wall reading (diffuse equilibrium at the wall velocity): the near-wall relation of
    // Eq. (NumerSana) keeps B of Eq. (CoeC) but has A = [(1+l)(1-r)(tau_s+1) + 2r(1+gamma)] / Den.
    // Matching the Kn term of the Poiseuille slip to Eq. (PhyscPoiSlip) (lambda = Kn H from
    // Eq. (tKnrela)) fixes A = (1 + gamma + L1 lambda) / (gamma + L1 lambda), i.e.
    // r / (1 - r) = (1 + l) k with k = (tau_s - gamma - L1 lambda) / (2 L1 lambda); along that
    // curve B is affine in 1 + l, B = B0 - 6 k (1 + l) / (tau_s + 2 k gamma), so matching the Kn^2
    // term (B = Bt) gives 1 + l in closed form.  k <= 0 has no admissible r (NaN, rejected).
    const double lam = (ts - 0.5) / sq;
    const double kw = (ts - g - L1 * lam) / (2.0 * L1 * lam);
    double l_raw;
    switch (a.l_mode) {
    case 2: l_raw = 0.0; break;
    case 3: l_raw = g; break;
    case 4: l_raw = 2.0 * g; break;
    case 5: l_raw = g * g; break;
    case 6: l_raw = g * g + g; break;
    case 7: l_raw = a.l_override; break;
    case 8: {
        const double tq = a.tau_q, nu = (ts - 0.5) / 3.0;
        const double at = (1.0 + g + L1 * lam) / (g + L1 * lam);
        const double bt = ((1.0 - at) * 2.0 * a.L2 * lam * lam + at * g * g - (1.0 + g) * (1.0 + g)) / (2.0 * nu);
        const double dd = ts + 2.0 * kw * g;
        const double b0 = ((1.0 + 2.0 * kw) * (1.0 + 4.0 * tq - 8.0 * ts - 8.0 * tq * ts) +
                           12.0 * kw * ((2.0 * g + 1.0) * t2 + (1.0 - 2.0 * g) * ts)) /
                          (2.0 * dd * t2);
        l_raw = kw > 0.0 ? (b0 - bt) * dd / (6.0 * kw) - 1.0 : __builtin_nan("");
        break;
    }
    default: l_raw = (sq * g * g + g * t2 * (L1 + sq)) / (sq * t2) + E; break;  // Eq. (Eqexlva)
    }
    double l = l_raw;
    if (a.l_mode == 0 && l_raw < -0.4) l = 0.0;
    if (a.l_mode == 1 && l_raw < 0.0) l = 0.0;
    double r;
    if (a.r_mode == 2) {
        r = a.r_override;
    } else if (a.r_mode == 3) {  // wall reading: A of the near-wall relation at the l used
        const double x = (1.0 + l) * kw;
        r = kw > 0.0 ? x / (1.0 + x) : __builtin_nan("");
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

// Streaming copy of n16 16-byte words (the copy that the step kernels' HBM traffic is compared with):
// a block moves 4 x 256 consecutive words, each thread issuing its four loads before its stores.
__global__ void __launch_bounds__(256) k_stream_copy(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                    uint64_t n16)
{
    const uint64_t base = uint64_t(blockIdx.x) * 1024u + threadIdx.x;
    uint4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t i = base + uint64_t(k) * 256u;
        if (i < n16) v[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t i = base + uint64_t(k) * 256u;
        if (i < n16) dst[i] = v[k];
    }
}

__global__ void __launch_bounds__(256) k_fill_zero_bytes(uint8_t* p, uint64_t n)
{
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// f_i(x, 0) = f_i^eq(rho, u - a/2) as the deviation w_i (rho - rho0) + w_i rho (3 c.v + 4.5 (c.v)^2
// - 1.5 v^2), v = u - a/2, stored where site x pulls it from: plane i at x - c_i, or the link
// array for populations that come from a wall.
template <typename T>
__global__ void __launch_bounds__(256) k_init_fields(const Geo g, T* pop, T* lnk, const double* rho_in,
                                                     const double* ux_in, const double* uy_in, double rho0,
                                                     double ax, double ay, double neq_tau)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const SiteLinks sl = site_links(g, s);
    const uint32_t fl = sl.fl, k0 = sl.k0;
    if (fl == kSolid) return;
    const Nbr b = neighbours(s, g.nx, g.ny);
    const double rho = rho_in[s];
    const double vx = ux_in[s] - 0.5 * ax, vy = uy_in[s] - 0.5 * ay;
    const double v2 = vx * vx + vy * vy;
    const uint64_t N = g.ps;
    // optional first-order non-equilibrium of the stress moments (neq_tau = tau_s > 0):
    // pxx = -(2/3) tau_s rho (d_x u_x - d_y u_y), pxy = -(1/3) tau_s rho (d_x u_y + d_y u_x), with the
    // derivatives taken from the fluid neighbours (central, one-sided next to a solid site, else 0);
    // f^neq = M^-1 (0, .., 0, pxx, pxy) gives +-pxx / 4 on the axis directions and +-pxy / 4 on the
    // diagonals
    double pxx = 0.0, pxy = 0.0;
    if (neq_tau > 0.0) {
        auto diff = [&](const double* f, uint32_t sp, uint32_t sm) {
            const bool fp = g.flags[sp] != kSolid, fm = g.flags[sm] != kSolid;
            return (fp && fm) ? (f[sp] - f[sm]) * 0.5 : (fp ? f[sp] - f[s] : (fm ? f[s] - f[sm] : 0.0));
        };
        const uint32_t e = b.row + b.xp, w = b.row + b.xm, nn = b.rowp + b.x, so = b.rowm + b.x;
        const double dxux = diff(ux_in, e, w), dyux = diff(ux_in, nn, so);
        const double dxuy = diff(uy_in, e, w), dyuy = diff(uy_in, nn, so);
        pxx = -(2.0 / 3.0) * neq_tau * rho * (dxux - dyuy);
        pxy = -(1.0 / 3.0) * neq_tau * rho * (dxuy + dyux);
    }
    const double qa = 0.25 * pxx, qd = 0.25 * pxy;
    auto dev = [&](double w, double cv, double nq) {
        return static_cast<T>(w * (rho - rho0) + w * rho * (3.0 * cv + 4.5 * cv * cv - 1.5 * v2) + nq);
    };
    auto put = [&](int i, int d, uint32_t up, T v) {
        if (fl & (1u << (d - 1)))
            lnk[k0 + rank_of(fl, d)] = v;
        else
            pop[i * N + up] = v;
    };
    pop[s] = dev(4.0 / 9.0, 0.0, 0.0);
    put(1, 3, b.row + b.xm, dev(1.0 / 9.0, vx, qa));
    put(2, 4, b.rowm + b.x, dev(1.0 / 9.0, vy, -qa));
    put(3, 1, b.row + b.xp, dev(1.0 / 9.0, -vx, qa));
    put(4, 2, b.rowp + b.x, dev(1.0 / 9.0, -vy, -qa));
    put(5, 7, b.rowm + b.xm, dev(1.0 / 36.0, vx + vy, qd));
    put(6, 8, b.rowm + b.xp, dev(1.0 / 36.0, -vx + vy, -qd));
    put(7, 5, b.rowp + b.xp, dev(1.0 / 36.0, -vx - vy, qd));
    put(8, 6, b.rowp + b.xm, dev(1.0 / 36.0, vx - vy, -qd));
}

template <typename T>
__global__ void __launch_bounds__(256) k_moments(const Geo g, const T* pop, const T* lnk, double* rho, double* ux,
                                                 double* uy, double rho0, double ax, double ay)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const SiteLinks sl = site_links(g, s);
    if (s >= g.n) return;
    if (sl.fl == kSolid) {
        rho[s] = 0.0;
        ux[s] = 0.0;
        uy[s] = 0.0;
        return;
    }
    const Nbr b = neighbours(s, g.nx, g.ny);
    const Pop<T> p = pull(pop, lnk, g.ps, s, b, sl.fl, sl.k0);
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

// Block-level fixed-order sum of three values over BLOCK threads; result valid in thread 0.
template <int BLOCK = kRedBlock>
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c)
{
    __shared__ double sh[3][BLOCK / 64];
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
        for (int i = 0; i < BLOCK / 64; ++i) {
            a += sh[0][i];
            b += sh[1][i];
            c += sh[2][i];
        }
    }
}

// Block-strided partial sums: sum |u - u_prev|^2, sum |u|^2, sum (rho - rho0) over fluid sites.
// The loop bound is block-uniform so that every lane takes part in the link prefix.
template <typename T>
__global__ void __launch_bounds__(kRedBlock) k_residual_partial(const ReduceArgs a)
{
    const T* pop = static_cast<const T*>(a.pop);
    const T* lnk = static_cast<const T*>(a.link);
    double s_du = 0.0, s_u = 0.0, s_dr = 0.0;
    const uint32_t stride = gridDim.x * kRedBlock;
    for (uint32_t base = blockIdx.x * kRedBlock; base < a.g.n; base += stride) {
        const uint32_t s = base + threadIdx.x;
        const SiteLinks sl = site_links(a.g, s);
        if (sl.fl == kSolid) continue;
        const Nbr b = neighbours(s, a.g.nx, a.g.ny);
        const Pop<T> p = pull(pop, lnk, a.g.ps, s, b, sl.fl, sl.k0);
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

// Batched residual partials: one active tile per loop trip, sums in a fixed order per tile.
template <typename T, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_residual_batch_partial(const BatchReduceArgs<T> a)
{
    const uint32_t ntile = *a.n_active;
    for (uint32_t t = blockIdx.x; t < ntile; t += gridDim.x) {
        const TileRef tr = a.tiles[t];
        const BatchInst<T> in = a.inst[tr.inst];
        const Geo g{a.flags + in.off, a.chunk_base + in.off / kChunk, in.n, in.nx, in.ny,
                    (in.n + kChunk - 1) / kChunk, a.ps};
        const uint32_t s = tr.start + threadIdx.x;
        const SiteLinks sl = site_links(g, s);
        double s_du = 0.0, s_u = 0.0, s_dr = 0.0;
        if (sl.fl != kSolid) {
            const Nbr b = neighbours(s, g.nx, g.ny);
            const Pop<T> p = pull(a.pop + in.off, a.link, g.ps, s, b, sl.fl, sl.k0);
            double dr, r, u, v;
            macro_fp64(p, static_cast<double>(in.ph.rho0), static_cast<double>(in.ph.ax),
                       static_cast<double>(in.ph.ay), dr, r, u, v);
            const double du = u - a.ux_prev[in.off + s], dv = v - a.uy_prev[in.off + s];
            s_du = du * du + dv * dv;
            s_u = u * u + v * v;
            s_dr = dr;
        }
        block_sum3<BLOCK>(s_du, s_u, s_dr);
        if (threadIdx.x == 0) {
            a.partial[3 * t + 0] = s_du;
            a.partial[3 * t + 1] = s_u;
            a.partial[3 * t + 2] = s_dr;
        }
        __syncthreads();
    }
}

// One block per active instance: fixed-order sum over its tiles.
__global__ void __launch_bounds__(kRedBlock) k_residual_batch_final(const double* partial, const uint32_t* tile_begin,
                                                                    double* out)
{
    const uint32_t i = blockIdx.x;
    const uint32_t t0 = tile_begin[i], t1 = tile_begin[i + 1];
    double x = 0.0, y = 0.0, z = 0.0;
    for (uint32_t t = t0 + threadIdx.x; t < t1; t += kRedBlock) {
        x += partial[3 * t + 0];
        y += partial[3 * t + 1];
        z += partial[3 * t + 2];
    }
    block_sum3(x, y, z);
    if (threadIdx.x == 0) {
        out[3 * i + 0] = x;
        out[3 * i + 1] = y;
        out[3 * i + 2] = z;
    }
}

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return static_cast<uint32_t>((a + b - 1) / b); }

template <typename T, int BLOCK>
hipError_t launch_step_block(const StepArgs<T>& a, bool write_u, bool node, hipStream_t stream)
{
    const uint32_t grid = ceil_div(a.g.n, BLOCK);
    const size_t lds = 5 * sizeof(T) * a.lds_links;
    if (write_u) {
        if (node)
            hipLaunchKernelGGL((k_step<T, true, true, BLOCK>), dim3(grid), dim3(BLOCK), lds, stream, a);
        else
            hipLaunchKernelGGL((k_step<T, true, false, BLOCK>), dim3(grid), dim3(BLOCK), lds, stream, a);
    } else {
        if (node)
            hipLaunchKernelGGL((k_step<T, false, true, BLOCK>), dim3(grid), dim3(BLOCK), lds, stream, a);
        else
            hipLaunchKernelGGL((k_step<T, false, false, BLOCK>), dim3(grid), dim3(BLOCK), lds, stream, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step_t(const StepArgs<T>& a, int block, bool write_u, bool node, hipStream_t stream)
{
    switch (block) {
    case 64: return launch_step_block<T, 64>(a, write_u, node, stream);
    case 128: return launch_step_block<T, 128>(a, write_u, node, stream);
    case 512: return launch_step_block<T, 512>(a, write_u, node, stream);
    case 1024: return launch_step_block<T, 1024>(a, write_u, node, stream);
    default: return launch_step_block<T, 256>(a, write_u, node, stream);
    }
}

template <typename T, int BLOCK>
hipError_t launch_batch_block(const BatchArgs<T>& a, uint32_t grid, bool write_u, bool node, hipStream_t stream)
{
    const size_t lds = 5 * sizeof(T) * a.lds_links;
    if (write_u) {
        if (node)
            hipLaunchKernelGGL((k_step_batch<T, true, true, BLOCK>), dim3(grid), dim3(BLOCK), lds, stream, a);
        else
            hipLaunchKernelGGL((k_step_batch<T, true, false, BLOCK>), dim3(grid), dim3(BLOCK), lds, stream, a);
    } else {
        if (node)
            hipLaunchKernelGGL((k_step_batch<T, false, true, BLOCK>), dim3(grid), dim3(BLOCK), lds, stream, a);
        else
            hipLaunchKernelGGL((k_step_batch<T, false, false, BLOCK>), dim3(grid), dim3(BLOCK), lds, stream, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_t(const BatchArgs<T>& a, int block, uint32_t grid, bool write_u, bool node,
                          hipStream_t stream)
{
    switch (block) {
    case 128: return launch_batch_block<T, 128>(a, grid, write_u, node, stream);
    case 512: return launch_batch_block<T, 512>(a, grid, write_u, node, stream);
    case 1024: return launch_batch_block<T, 1024>(a, grid, write_u, node, stream);
    default: return launch_batch_block<T, 256>(a, grid, write_u, node, stream);
    }
}

template <typename T>
hipError_t launch_residual_batch_t(const BatchReduceArgs<T>& a, int block, uint32_t grid,
                                   const uint32_t* tile_begin, uint32_t n_inst, double* out, hipStream_t stream)
{
    switch (block) {
    case 128: hipLaunchKernelGGL((k_residual_batch_partial<T, 128>), dim3(grid), dim3(128), 0, stream, a); break;
    case 512: hipLaunchKernelGGL((k_residual_batch_partial<T, 512>), dim3(grid), dim3(512), 0, stream, a); break;
    case 1024: hipLaunchKernelGGL((k_residual_batch_partial<T, 1024>), dim3(grid), dim3(1024), 0, stream, a); break;
    default: hipLaunchKernelGGL((k_residual_batch_partial<T, 256>), dim3(grid), dim3(256), 0, stream, a); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_inst == 0) return e;
    hipLaunchKernelGGL(k_residual_batch_final, dim3(n_inst), dim3(kRedBlock), 0, stream, a.partial, tile_begin, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step_batch_f64(const BatchArgs<double>& a, int block, uint32_t grid, bool write_u, bool node,
                                 hipStream_t stream)
{
    return launch_batch_t<double>(a, block, grid, write_u, node, stream);
}

hipError_t launch_step_batch_f32(const BatchArgs<float>& a, int block, uint32_t grid, bool write_u, bool node,
                                 hipStream_t stream)
{
    return launch_batch_t<float>(a, block, grid, write_u, node, stream);
}

hipError_t launch_residual_batch_f64(const BatchReduceArgs<double>& a, int block, uint32_t grid,
                                     const uint32_t* tile_begin, uint32_t n_inst, double* out, hipStream_t stream)
{
    return launch_residual_batch_t<double>(a, block, grid, tile_begin, n_inst, out, stream);
}

hipError_t launch_residual_batch_f32(const BatchReduceArgs<float>& a, int block, uint32_t grid,
                                     const uint32_t* tile_begin, uint32_t n_inst, double* out, hipStream_t stream)
{
    return launch_residual_batch_t<float>(a, block, grid, tile_begin, n_inst, out, stream);
}

size_t step_lds_bytes(bool fp32, uint32_t max_links) { return 5 * (fp32 ? 4 : 8) * size_t(max_links); }

size_t step2_lds_bytes(bool fp32, int rows, uint32_t max_links)
{
    const size_t t = fp32 ? 4 : 8;
    return t * (9 * size_t(rows + 2) * (kFuseTX + 2) + 5 * size_t(max_links)) + 4 * size_t(max_links) +
           5 * size_t(rows) * kFuseTX;
}

namespace {

template <typename T, int TY, int RPW>
hipError_t launch_step2_rows(const StepArgs<T>& a, bool write_u, bool node, hipStream_t stream)
{
    const uint32_t grid = (a.g.nx / kFuseTX) * (a.g.ny / TY);
    const size_t lds = step2_lds_bytes(sizeof(T) == 4, TY, a.lds_links);
    const dim3 block(step2_threads<TY, RPW>());
    if (write_u) {
        if (node)
            hipLaunchKernelGGL((k_step2<T, true, true, TY, RPW>), dim3(grid), block, lds, stream, a);
        else
            hipLaunchKernelGGL((k_step2<T, true, false, TY, RPW>), dim3(grid), block, lds, stream, a);
    } else {
        if (node)
            hipLaunchKernelGGL((k_step2<T, false, true, TY, RPW>), dim3(grid), block, lds, stream, a);
        else
            hipLaunchKernelGGL((k_step2<T, false, false, TY, RPW>), dim3(grid), block, lds, stream, a);
    }
    return hipGetLastError();
}

}  // namespace

// fp64: one LDS row per step-1 wave (on 8-row tiles LDS and registers already limit a CU to two
// blocks); fp32: two rows per wave, so that eight 4-wave blocks of 4-row tiles share a CU and each
// lane has two sites' loads in flight.
hipError_t launch_step2_f64(const StepArgs<double>& a, int rows, bool write_u, bool node, hipStream_t stream)
{
    return rows == 4 ? launch_step2_rows<double, 4, 1>(a, write_u, node, stream)
                     : launch_step2_rows<double, 8, 1>(a, write_u, node, stream);
}

hipError_t launch_step2_f32(const StepArgs<float>& a, int rows, bool write_u, bool node, hipStream_t stream)
{
    return rows == 4 ? launch_step2_rows<float, 4, 2>(a, write_u, node, stream)
                     : launch_step2_rows<float, 8, 2>(a, write_u, node, stream);
}

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

hipError_t launch_stream_copy(void* dst, const void* src, uint64_t bytes, hipStream_t stream)
{
    const uint64_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stream_copy, dim3(ceil_div(n16, 1024)), dim3(256), 0, stream, static_cast<uint4*>(dst),
                       static_cast<const uint4*>(src), n16);
    return hipGetLastError();
}

hipError_t launch_init_fields(bool fp32, const Geo& g, void* pop, void* link, const double* rho, const double* ux,
                              const double* uy, double rho0, double ax, double ay, double neq_tau, hipStream_t stream)
{
    const dim3 grid(ceil_div(g.n, 256)), blk(256);
    if (fp32)
        hipLaunchKernelGGL(k_init_fields<float>, grid, blk, 0, stream, g, static_cast<float*>(pop),
                           static_cast<float*>(link), rho, ux, uy, rho0, ax, ay, neq_tau);
    else
        hipLaunchKernelGGL(k_init_fields<double>, grid, blk, 0, stream, g, static_cast<double*>(pop),
                           static_cast<double*>(link), rho, ux, uy, rho0, ax, ay, neq_tau);
    return hipGetLastError();
}

hipError_t launch_moments(bool fp32, const Geo& g, const void* pop, const void* link, double* rho, double* ux,
                          double* uy, double rho0, double ax, double ay, hipStream_t stream)
{
    const dim3 grid(ceil_div(g.n, 256)), blk(256);
    if (fp32)
        hipLaunchKernelGGL(k_moments<float>, grid, blk, 0, stream, g, static_cast<const float*>(pop),
                           static_cast<const float*>(link), rho, ux, uy, rho0, ax, ay);
    else
        hipLaunchKernelGGL(k_moments<double>, grid, blk, 0, stream, g, static_cast<const double*>(pop),
                           static_cast<const double*>(link), rho, ux, uy, rho0, ax, ay);
    return hipGetLastError();
}

uint32_t residual_blocks(uint32_t n)
{
    const uint32_t b = ceil_div(n, kRedBlock);
    return b < kRedMaxBlocks ? (b == 0 ? 1u : b) : kRedMaxBlocks;
}

hipError_t launch_residual(bool fp32, const ReduceArgs& a, double* out, hipStream_t stream)
{
    const uint32_t nb = residual_blocks(a.g.n);
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
