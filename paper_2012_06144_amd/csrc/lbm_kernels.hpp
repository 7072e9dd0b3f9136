// Fused stream-collide sweeps of the coupled phase-field / hydrodynamic
// lattice Boltzmann step (Holzer et al., IJHPCA 2020) for gfx950.
//
// Memory layout (all in the caller-provided workspace):
//   PDF sets: blocked structure of arrays.  Cells are grouped in blocks of
//   kB = 512 consecutive cells (x fastest); a block stores its q directions
//   one after another, each as kB contiguous values, so a wavefront reads
//   or writes 256-byte runs and all q runs of one block share a few DRAM
//   pages.  Two copies per set (source / destination, swapped every step).
//   Both sets hold POST-collision populations at the cell; both sweeps
//   pull-stream (read direction i from the neighbour at x - e_i), which on
//   gfx950 costs nothing over aligned access while push writes to
//   neighbours do not.
//   phi: two planes (previous / new); u: three planes.
// One thread updates one cell; blocks of 256 threads cover consecutive
// cells.  Block indices are remapped so that each of the 8 XCDs of the
// MI355X works on one contiguous slab of the grid, which keeps the phase
// field rows a cell's stencil re-reads inside that XCD's L2.
#pragma once

#include "lbm_lattice.hpp"

namespace lbm {

#ifndef LBM_BLOCK
#define LBM_BLOCK 256
#endif
#ifndef LBM_LOGB
#define LBM_LOGB 9
#endif
#ifndef LBM_FASTDIV
#define LBM_FASTDIV 1
#endif
constexpr int kBlock = LBM_BLOCK;  // threads per block of the sweeps
constexpr int kXcds = 8;
constexpr int kLogB = LBM_LOGB;    // cells per PDF block = 512
constexpr int kB = 1 << kLogB;

// Storage index of direction q of cell c in a blocked PDF set with Q directions.
template <int Q>
__host__ __device__ inline int64_t pidx(int q, int c)
{
    return ((int64_t)(c >> kLogB) * Q + q) * kB + (c & (kB - 1));
}
constexpr int kRedBlocks = 1024;  // fixed grid of the deterministic reductions
constexpr int kRedVals = 12;      // 11 sums + 1 max

// Physical constants of one launch, in the sweep's arithmetic type.
template <class R>
struct Phys {
    R phi_L, phi_H, phi_0, inv_dphi;     // inv_dphi = 1/(phi_H - phi_L)
    R phi_lo, phi_hi;                    // min and max of phi_L, phi_H
    R xi, inv_xi, omega_phi;             // interface width, its inverse, phase-field relaxation rate
    R rho_L, drho;                       // drho = rho_H - rho_L
    R tau_L, dtau;                       // dtau = tau_H - tau_L
    R beta, kappa;                       // 12 sigma/xi, 3 sigma xi/2
    R accel[3];
    R rho_ref;                           // F_b = (rho - rho_ref) accel
    R normal_eps;
};

// Density and relaxation time of a cell (eq. density, tau interpolation of
// Sec. 3.2), linear in phi between the bulk phases.  By default phi is
// clamped to [phi_L, phi_H] first: the phase field overshoots that interval
// by ~1e-3 in the cores of small bubbles, and at rho_H/rho_L = 1000 an
// undershoot of 1e-3 would put rho near zero.  With the literal
// interpolation the clamp bounds are +-max and the clamp does nothing.
template <class R>
__host__ __device__ inline R phase_clamp(const Phys<R> &ph, R phi)
{
    return phi < ph.phi_lo ? ph.phi_lo : (phi > ph.phi_hi ? ph.phi_hi : phi);
}
template <class R>
__host__ __device__ inline R density_of(const Phys<R> &ph, R phi)
{
    return ph.rho_L + (phase_clamp(ph, phi) - ph.phi_L) * ph.drho * ph.inv_dphi;
}

// Division by a run-time invariant d >= 1 with a multiply-high and shifts
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994, Fig. 4.1): q = (t + ((n - t) >> 1)) >> (l - 1),
// t = mulhi(m, n), l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1.
struct FastDiv {
    uint32_t d, m, l;
    __host__ __device__ uint32_t div(uint32_t n) const
    {
        if (l == 0) return n;
        const uint32_t t = (uint32_t)(((uint64_t)m * n) >> 32);
        return (t + ((n - t) >> 1)) >> (l - 1);
    }
};

inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f{d, 0u, 0u};
    uint32_t l = 0;
    while (((uint64_t)1 << l) < d) ++l;
    f.l = l;
    if (l > 0) f.m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
    return f;
}

struct Grid {
    int nx, ny, nz;
    int walls;
    int ncells;
    int half;        // ceil(ncells / 2): paired 16-bit storage keeps cells c and c + half in one word
    int64_t fplane;  // field plane stride (elements) of u
    FastDiv dnx, dny;
};

// Logical block index: block b runs on XCD b % 8 (round-robin dispatch);
// give XCD k the k-th contiguous share of the logical blocks.
__device__ inline int xcd_block()
{
    const int b = blockIdx.x, G = gridDim.x;
    const int xcd = b % kXcds, idx = b / kXcds;
    const int q = G / kXcds, r = G % kXcds;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Neighbour offsets of one cell (relative element offsets inside a plane).
struct Nbr {
    int xm, xp, ym, yp, zm, zp;
    bool wm, wp;  // y-1 / y+1 is a wall row
    __device__ int off(int dx, int dy, int dz) const
    {
        return (dx < 0 ? xm : dx > 0 ? xp : 0) + (dy < 0 ? ym : dy > 0 ? yp : 0) +
               (dz < 0 ? zm : dz > 0 ? zp : 0);
    }
    // Phase-field stencil offset: a wall row is read at its mirror image,
    // which is the current row.
    __device__ int offm(int dx, int dy, int dz) const
    {
        return (dx < 0 ? xm : dx > 0 ? xp : 0) + (dy < 0 ? (wm ? 0 : ym) : dy > 0 ? (wp ? 0 : yp) : 0) +
               (dz < 0 ? zm : dz > 0 ? zp : 0);
    }
};

__device__ inline bool decode(const Grid &g, int c, int &x, int &y, int &z, Nbr &n)
{
#if LBM_FASTDIV
    const int t = (int)g.dnx.div((uint32_t)c);
    x = c - t * g.nx;
    z = (int)g.dny.div((uint32_t)t);
    y = t - z * g.ny;
#else
    x = c % g.nx;
    const int t = c / g.nx;
    y = t % g.ny;
    z = t / g.ny;
#endif
    if (g.walls && (y == 0 || y == g.ny - 1)) return false;
    const int nxy = g.nx * g.ny;
    n.xm = (x == 0) ? g.nx - 1 : -1;
    n.xp = (x == g.nx - 1) ? -(g.nx - 1) : 1;
    if (g.walls) {
        n.ym = -g.nx;
        n.yp = g.nx;
        n.wm = (y == 1);
        n.wp = (y == g.ny - 2);
    } else {
        n.ym = (y == 0) ? (g.ny - 1) * g.nx : -g.nx;
        n.yp = (y == g.ny - 1) ? -(g.ny - 1) * g.nx : g.nx;
        n.wm = n.wp = false;
    }
    n.zm = (z == 0) ? (g.nz - 1) * nxy : -nxy;
    n.zp = (z == g.nz - 1) ? -(g.nz - 1) * nxy : nxy;
    return true;
}

// x / c_s^2.  FP64 divides by the rounded 1/3 exactly as a literal reading of
// the formulas does; FP32 multiplies by 3.
__device__ inline double by_cs2(double v) { return v / (1.0 / 3.0); }
__device__ inline float by_cs2(float v) { return v * 3.0f; }
template <class R>
__device__ inline R cs2() { return R(1) / R(3); }

// Gamma_i(u) = w_i [1 + e.u/cs^2 + (e.u)^2/(2 cs^4) - u.u/(2 cs^2)] (Sec. 3.1)
template <int Q, class R>
__device__ inline R gamma_i(int i, R ux, R uy, R uz, R uu)
{
    const R eu = R(ev<Q>(i, 0)) * ux + R(ev<Q>(i, 1)) * uy + R(ev<Q>(i, 2)) * uz;
    if constexpr (std::is_same<R, float>::value) {
        // 1/(2 cs^4) = 4.5 and 1/(2 cs^2) = 1.5 exactly: multiplications, where
        // a division by the rounded constants costs ~10 VALU instructions each
        return wgt<Q, R>(i) * (R(1) + by_cs2(eu) + (eu * eu) * R(4.5) - uu * R(1.5));
    } else {
        const R c2 = cs2<R>();
        return wgt<Q, R>(i) * (R(1) + by_cs2(eu) + (eu * eu) / (R(2) * c2 * c2) - uu / (R(2) * c2));
    }
}

// Hydrodynamic equilibrium g_eq_i = p* w_i + (Gamma_i - w_i) (Sec. 3.2), with
// the w_i of Gamma cancelled algebraically so small g are not formed as a
// difference of O(w) numbers.
template <int Q, class R>
__device__ inline R geq_i(int i, R ps, R ux, R uy, R uz, R uu)
{
    const R eu = R(ev<Q>(i, 0)) * ux + R(ev<Q>(i, 1)) * uy + R(ev<Q>(i, 2)) * uz;
    if constexpr (std::is_same<R, float>::value) {
        return wgt<Q, R>(i) * (ps + by_cs2(eu) + (eu * eu) * R(4.5) - uu * R(1.5));
    } else {
        const R c2 = cs2<R>();
        return wgt<Q, R>(i) * (ps + by_cs2(eu) + (eu * eu) / (R(2) * c2 * c2) - uu / (R(2) * c2));
    }
}

// Previous / new phase field around a cell, as the stencils read it (wall
// rows mirrored onto the current row).  PhiG reads global memory; PhiL reads
// the three LDS planes a z-marching block keeps.
template <class R>
struct PhiG {
    const R *__restrict__ phi;
    int c;
    const Nbr *n;
    __device__ R at(int dx, int dy, int dz) const { return phi[c + n->offm(dx, dy, dz)]; }
};

#ifndef LBM_ZMARCH
#define LBM_ZMARCH 0  // 1: sweeps march in z with the phase field staged in LDS
#endif
#ifndef LBM_ZM_TX
#define LBM_ZM_TX 64
#endif
constexpr int kTX = LBM_ZM_TX, kTY = LBM_BLOCK / LBM_ZM_TX;  // z-marching tile, one thread per cell
constexpr int kZmBlocks = 8192;            // target block count of a z-marching launch
static_assert(kTX * kTY == LBM_BLOCK, "a z-marching tile has one thread per cell");
constexpr int kLX = kTX + 2, kLY = kTY + 2;

template <class R>
struct PhiL {
    const R *pl[3];  // planes z-1, z, z+1: (kTY+2) rows of (kTX+2) values, halo included
    int o;           // (ty+1) kLX + (tx+1)
    __device__ R at(int dx, int dy, int dz) const { return pl[dz + 1][o + dy * kLX + dx]; }
};

// Isotropic gradient (eq. grad) as antisymmetric pair differences over the
// half set, and (optionally) Laplacian (eq. lap), on phi with the wall mirror.
template <int Q, class R, bool LAP, class P>
__device__ inline void stencil(const P &phi, R grad[3], R &lap)
{
    R acc[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const int dx = ev<Q>(i, 0), dy = ev<Q>(i, 1), dz = ev<Q>(i, 2);
        const R d = phi.at(dx, dy, dz) - phi.at(-dx, -dy, -dz);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int ea = ev<Q>(i, a);
            if (ea > 0) acc[a] += wgt<Q, R>(i) * d;
            if (ea < 0) acc[a] -= wgt<Q, R>(i) * d;
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) grad[a] = by_cs2(acc[a]);
    if (LAP) {
        const R pc = phi.at(0, 0, 0);
        R s = R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int dx = ev<Q>(i, 0), dy = ev<Q>(i, 1), dz = ev<Q>(i, 2);
            s += wgt<Q, R>(i) * (phi.at(dx, dy, dz) - pc);
        }
        lap = R(2) * by_cs2(s);
    }
}

template <class S>
struct SweepArgs {
    const typename S::pdf_t *__restrict__ src;
    typename S::pdf_t *__restrict__ dst;
    const typename S::real *__restrict__ phi_in;
    typename S::real *__restrict__ phi_out;
    typename S::real *__restrict__ u;
    Grid g;
    Phys<typename S::real> ph;
};

// Element index of population q of cell c in a PDF buffer of storage S.
// 16-bit storage is paired: cells c and c + half (half = ceil(N/2); for even
// nz, (x, y, z) and (x, y, z + nz/2)) share the 32-bit word at the blocked
// index of the lower cell, the lower cell in the low half.
template <class S, int Q>
__device__ inline int64_t pdf_index(int q, int c, const Grid &g)
{
    if constexpr (S::paired) {
        const int h = c >= g.half ? 1 : 0;
        return 2 * pidx<Q>(q, c - h * g.half) + h;
    } else {
        return pidx<Q>(q, c);
    }
}

// Storage index of the population of direction i arriving at cell c: the
// post-collision value of the upstream cell c - e_i or, when that cell is a
// wall, the value of the opposite direction at c itself (halfway
// bounce-back: what left c towards the wall comes back reversed).
template <class S, int Q>
__device__ inline int64_t pull_idx(int i, int c, const Nbr &n, const Grid &g)
{
    const int dx = ev<Q>(i, 0), dy = ev<Q>(i, 1), dz = ev<Q>(i, 2);
    const bool bb = (dy > 0 && n.wm) || (dy < 0 && n.wp);
    return bb ? pdf_index<S, Q>(opp(i), c, g) : pdf_index<S, Q>(i, c + n.off(-dx, -dy, -dz), g);
}

// Population I/O of the per-cell sweep bodies.  IOGlobal pulls from and
// stores to global memory for one cell; IORegs reads and writes register
// arrays that a paired kernel fills from and drains to 32-bit words.
template <class S, int Q>
struct IOGlobal {
    const typename S::pdf_t *__restrict__ src;
    typename S::pdf_t *__restrict__ dst;
    int c;
    const Nbr *n;
    const Grid *g;
    __device__ typename S::pdf_t load(int i) const { return ld_stream(src + pull_idx<S, Q>(i, c, *n, *g)); }
    __device__ void store(int i, typename S::pdf_t v) const { st_stream(dst + pdf_index<S, Q>(i, c, *g), v); }
};

template <class S, int Q>
struct IORegs {
    const typename S::pdf_t *in;
    typename S::pdf_t *out;
    __device__ typename S::pdf_t load(int i) const { return in[i]; }
    __device__ void store(int i, typename S::pdf_t v) const { out[i] = v; }
};

// ---- phase-field sweep: pull-stream h, phi = sum h (eq. updatePhaseField),
// normal and theta from the previous phi (eqs. allen_cahn, grad), forcing
// (eq. interfaceTracking), equilibrium phi Gamma(u), single-rate collision
// (eq. lb_interface); store post-collision h at the cell ----------------------
// PHI_OUT = false: the collision step of the straightforward algorithm, whose
// phase field was already written by a pass of its own.
template <class S, class P, class IO, bool U_REG = false, bool PHI_OUT = true>
__device__ inline void phase_cell(const SweepArgs<S> &a, int c, const Nbr &n, const P &phiA, const IO &io,
                                  const typename S::real *u_reg = nullptr)
{
    using R = typename S::real;
    constexpr int QP = S::QP;
    // previous phase field at x + e_i (stencil points of the phase-field set; wall rows mirrored)
    R phs[QP];
#pragma unroll
    for (int i = 0; i < QP; ++i) phs[i] = phiA.at(ev<QP>(i, 0), ev<QP>(i, 1), ev<QP>(i, 2));

    // The population arrives from x - e_i (phs[opp(i)]) or bounces back at x.
    // The FP32 and 16-bit paths keep the phi budget of the cell in FP64: the
    // decoded populations are summed exactly, so sum(phi) moves only by the
    // single rounding of the rest population below.
    R Pi[QP];
    double phi_acc = 0.0;
#pragma unroll
    for (int i = 0; i < QP; ++i) {
        const bool bb = (ev<QP>(i, 1) > 0 && n.wm) || (ev<QP>(i, 1) < 0 && n.wp);
        const typename S::pdf_t v = io.load(i);
        const R up = bb ? phs[0] : phs[opp(i)];
        if constexpr (std::is_same<R, double>::value) {
            Pi[i] = dec_h<S>(v, up, i);
            phi_acc += Pi[i];
        } else {
            const double p64 = dec_h64<S>(v, up, i);
            Pi[i] = R(p64);
            phi_acc += p64;
        }
    }
    const R phi = R(phi_acc);
    if constexpr (PHI_OUT) st_field(a.phi_out + c, phi);

    // isotropic gradient (eq. grad) from antisymmetric pairs of the half set
    R acc[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 1; i < QP; i += 2) {
        const R d = phs[i] - phs[i + 1];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (ev<QP>(i, k) > 0) acc[k] += wgt<QP, R>(i) * d;
            if (ev<QP>(i, k) < 0) acc[k] -= wgt<QP, R>(i) * d;
        }
    }
    R grad[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) grad[k] = by_cs2(acc[k]);
    const R gn = sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]);
    R nrm[3];
    const R dp = phs[0] - a.ph.phi_0;
    R theta;
    if constexpr (std::is_same<R, float>::value) {
        const R inv = R(1) / (gn + a.ph.normal_eps);
#pragma unroll
        for (int k = 0; k < 3; ++k) nrm[k] = grad[k] * inv;
        theta = (R(1) - R(4) * dp * dp) * a.ph.inv_xi;
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) nrm[k] = grad[k] / (gn + a.ph.normal_eps);
        theta = (R(1) - R(4) * dp * dp) / a.ph.xi;
    }

    // u of the cell: from memory, or (U_REG) from the registers of a fused hydrodynamic sweep that just wrote it
    R ux, uy, uz;
    if constexpr (U_REG) {
        ux = u_reg[0];
        uy = u_reg[1];
        uz = u_reg[2];
    } else {
        ux = a.u[c];
        uy = a.u[a.g.fplane + c];
        uz = a.u[2 * a.g.fplane + c];
    }
    const R uu = ux * ux + uy * uy + uz * uz;
    const R om = a.ph.omega_phi;
    R hs[QP];
    if constexpr (!S::phase_mrt) {
#pragma unroll
        for (int i = 0; i < QP; ++i) {
            const R en = R(ev<QP>(i, 0)) * nrm[0] + R(ev<QP>(i, 1)) * nrm[1] + R(ev<QP>(i, 2)) * nrm[2];
            const R F = theta * wgt<QP, R>(i) * en;
            const R heq = phi * gamma_i<QP, R>(i, ux, uy, uz, uu);
            hs[i] = Pi[i] + om * (heq - Pi[i] - R(0.5) * F) + F;
        }
    } else {
        // Raw-moment MRT (Sec. 3.1): the first-order moments relax with
        // omega, every other moment with one.  With the monomial moment set
        // the first-order columns of the inverse moment matrix are
        // (delta_{+k} - delta_{-k})/2 on the axis pair of direction k, so
        // h* = h_eq + F/2 + (omega - 1)/2 (+-) j_k(h_eq - h - F/2) on the
        // six axis populations and h_eq + F/2 on all others.
        R d[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int i = 0; i < QP; ++i) {
            const R en = R(ev<QP>(i, 0)) * nrm[0] + R(ev<QP>(i, 1)) * nrm[1] + R(ev<QP>(i, 2)) * nrm[2];
            const R F = theta * wgt<QP, R>(i) * en;
            const R heq = phi * gamma_i<QP, R>(i, ux, uy, uz, uu);
            const R di = heq - Pi[i] - R(0.5) * F;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (ev<QP>(i, k) > 0) d[k] += di;
                if (ev<QP>(i, k) < 0) d[k] -= di;
            }
            hs[i] = heq + R(0.5) * F;
        }
        const R hw = R(0.5) * (om - R(1));
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            hs[1 + 2 * k] += hw * d[k];
            hs[2 + 2 * k] -= hw * d[k];
        }
    }
    if constexpr (std::is_same<R, double>::value) {
#pragma unroll
        for (int i = 0; i < QP; ++i) io.store(i, enc_h<S>(hs[i], phi, i));
    } else {
        // The collision conserves phi exactly; in FP32 the rounded weights do
        // not sum to one and 16-bit storage rounds every population, which
        // would bias sum(phi) every step.  Close the budget on the rest
        // population, using the values the next sweep will decode.
        double rest = phi_acc;
#pragma unroll
        for (int i = 1; i < QP; ++i) {
            const typename S::pdf_t v = enc_h<S>(hs[i], phi, i);
            rest -= dec_h64<S>(v, phi, i);
            io.store(i, v);
        }
        io.store(0, enc_h64<S>(rest, phi, 0));
    }
}

template <class S>
__global__ __launch_bounds__(kBlock) void k_phase(const SweepArgs<S> a)
{
    const int c = xcd_block() * kBlock + threadIdx.x;
    if (c >= a.g.ncells) return;
    int x, y, z;
    Nbr n;
    if (!decode(a.g, c, x, y, z, n)) return;
    phase_cell<S>(a, c, n, PhiG<typename S::real>{a.phi_in, c, &n}, IOGlobal<S, S::QP>{a.src, a.dst, c, &n, &a.g});
}

// ---- hydrodynamic sweep: pull-stream g, moments, forces from the new phi
// (eqs. forceHydro, pressure_force, surfaceTension, chemPot, viscousForce and
// buoyancy), velocity update (eq. updateVelocityField), moment-space
// collision (eq. improved_collision) in closed form; store post-collision g
// at the cell ------------------------------------------------------------------
//
// Closed form of the collision: with a weighted-orthogonal moment basis, the
// six second-order moments relaxed with s and all others with 1, and the
// force on the first-order moments only,
//   g*_i = g_eq_i(p*, u) + F_i/2 + (1 - s) w_i/(2 cs^4) (e_i e_i - cs^2 I) : A,
//   A = Pi - p* cs^2 I - u u^T,  F_i = w_i e_i.F/(rho cs^2),
// and the bracket of the viscous force is s A(u_old).
//
// HMODE selects the steps of the body: kHydroFull (velocity update and
// collision, the fused step), kHydroUpdateU (velocity update only) or
// kHydroCollide (collision only, with the stored velocity both in the
// viscous force and in the equilibrium) -- the last two are separate passes
// of the straightforward algorithm.
constexpr int kHydroFull = 0, kHydroUpdateU = 1, kHydroCollide = 2;
template <class S, class P, class IO, bool U_OUT = false, int HMODE = kHydroFull>
__device__ inline void hydro_cell(const SweepArgs<S> &a, int c, const Nbr &n, const P &phiB, const IO &io,
                                  typename S::real *u_new = nullptr)
{
    using R = typename S::real;
    constexpr int QH = S::QH;
    static_assert(!S::lowp || QH == 27, "16-bit storage keeps the D3Q27 hydrodynamic set");
    R ps = R(0), j[3] = {R(0), R(0), R(0)};
    R Pxx = R(0), Pyy = R(0), Pzz = R(0), Pxy = R(0), Pxz = R(0), Pyz = R(0);
    if constexpr (S::lowp) {
        // g_i = w_i x stored_i / kScale: sum the stored values per weight
        // class (rest, axis, edge, corner) and apply each class weight once
        R m[4][10];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int q = 0; q < 10; ++q) m[k][q] = R(0);
#pragma unroll
        for (int i = 0; i < QH; ++i) {
            const R v = S::raw_ld(io.load(i));
            const int ex = ev<QH>(i, 0), ey = ev<QH>(i, 1), ez = ev<QH>(i, 2), k = l1<QH>(i);
            m[k][0] += v;
            if (ex) m[k][1] += ex > 0 ? v : -v;
            if (ey) m[k][2] += ey > 0 ? v : -v;
            if (ez) m[k][3] += ez > 0 ? v : -v;
            if (ex) m[k][4] += v;
            if (ey) m[k][5] += v;
            if (ez) m[k][6] += v;
            if (ex && ey) m[k][7] += (ex * ey > 0) ? v : -v;
            if (ex && ez) m[k][8] += (ex * ez > 0) ? v : -v;
            if (ey && ez) m[k][9] += (ey * ez > 0) ? v : -v;
        }
        R mom[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            mom[q] = R(0);
#pragma unroll
            for (int k = 0; k < 4; ++k) mom[q] += m[k][q] * (class_w27<R>(k) * (R(1) / R(S::kScale)));
        }
        ps = mom[0];
        j[0] = mom[1];
        j[1] = mom[2];
        j[2] = mom[3];
        Pxx = mom[4];
        Pyy = mom[5];
        Pzz = mom[6];
        Pxy = mom[7];
        Pxz = mom[8];
        Pyz = mom[9];
    } else {
#pragma unroll
        for (int i = 0; i < QH; ++i) {
            const R gi = dec_g<S>(io.load(i), i);
            const int ex = ev<QH>(i, 0), ey = ev<QH>(i, 1), ez = ev<QH>(i, 2);
            ps += gi;
            if (ex) j[0] += ex > 0 ? gi : -gi;
            if (ey) j[1] += ey > 0 ? gi : -gi;
            if (ez) j[2] += ez > 0 ? gi : -gi;
            if (ex) Pxx += gi;
            if (ey) Pyy += gi;
            if (ez) Pzz += gi;
            if (ex && ey) Pxy += (ex * ey > 0) ? gi : -gi;
            if (ex && ez) Pxz += (ex * ez > 0) ? gi : -gi;
            if (ey && ez) Pyz += (ey * ez > 0) ? gi : -gi;
        }
    }

    const R phi = phiB.at(0, 0, 0);
    R grad[3], lap;
    stencil<QH, R, true>(phiB, grad, lap);

    const Phys<R> &ph = a.ph;
    const R rho = density_of(ph, phi);
    const R tau = ph.tau_L + (phase_clamp(ph, phi) - ph.phi_L) * ph.dtau * ph.inv_dphi;
    const R s = R(1) / (tau + R(0.5));
    const R nu = tau * cs2<R>();
    R grho[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) grho[k] = ph.drho * ph.inv_dphi * grad[k];
    const R mu = R(4) * ph.beta * (phi - ph.phi_L) * (phi - ph.phi_H) * (phi - ph.phi_0) - ph.kappa * lap;

    const R c2 = cs2<R>();
    const R uox = a.u[c], uoy = a.u[a.g.fplane + c], uoz = a.u[2 * a.g.fplane + c];
    // A(u_old) = Pi - p* cs^2 I - u_old u_old^T; viscous bracket = s A
    const R Axx = Pxx - ps * c2 - uox * uox, Ayy = Pyy - ps * c2 - uoy * uoy, Azz = Pzz - ps * c2 - uoz * uoz;
    const R Axy = Pxy - uox * uoy, Axz = Pxz - uox * uoz, Ayz = Pyz - uoy * uoz;
    const R vf = std::is_same<R, float>::value ? -tau * s : -nu / c2 * s;  // nu / cs^2 = tau
    const R rb = rho - ph.rho_ref;
    R F[3];
    F[0] = -ps * c2 * grho[0] + mu * grad[0] + vf * (Axx * grho[0] + Axy * grho[1] + Axz * grho[2]) +
           rb * ph.accel[0];
    F[1] = -ps * c2 * grho[1] + mu * grad[1] + vf * (Axy * grho[0] + Ayy * grho[1] + Ayz * grho[2]) +
           rb * ph.accel[1];
    F[2] = -ps * c2 * grho[2] + mu * grad[2] + vf * (Axz * grho[0] + Ayz * grho[1] + Azz * grho[2]) +
           rb * ph.accel[2];

    R ux, uy, uz;
    R inv_rho = R(0);
    if constexpr (std::is_same<R, float>::value) inv_rho = R(1) / rho;
    if constexpr (HMODE == kHydroCollide) {
        ux = uox;
        uy = uoy;
        uz = uoz;
    } else {
        if constexpr (std::is_same<R, float>::value) {
            const R h = R(0.5) * inv_rho;
            ux = j[0] + F[0] * h;
            uy = j[1] + F[1] * h;
            uz = j[2] + F[2] * h;
        } else {
            ux = j[0] + F[0] / (R(2) * rho);
            uy = j[1] + F[1] / (R(2) * rho);
            uz = j[2] + F[2] / (R(2) * rho);
        }
        st_field(a.u + c, ux);
        st_field(a.u + a.g.fplane + c, uy);
        st_field(a.u + 2 * a.g.fplane + c, uz);
    }
    if constexpr (HMODE == kHydroUpdateU) return;
    if constexpr (U_OUT) {
        u_new[0] = ux;
        u_new[1] = uy;
        u_new[2] = uz;
    }

    const R uu = ux * ux + uy * uy + uz * uz;
    const R Bxx = Pxx - ps * c2 - ux * ux, Byy = Pyy - ps * c2 - uy * uy, Bzz = Pzz - ps * c2 - uz * uz;
    const R Bxy = Pxy - ux * uy, Bxz = Pxz - ux * uz, Byz = Pyz - uy * uz;
    const R trB = Bxx + Byy + Bzz;
    const R neq = std::is_same<R, float>::value ? (R(1) - s) * R(4.5) : (R(1) - s) / (R(2) * c2 * c2);
    const R finv = std::is_same<R, float>::value ? R(3) * inv_rho : R(1) / (rho * c2);
    if constexpr (std::is_same<R, float>::value) {
        // g*_i / w_i = (p* - 1.5 u.u) + e.u (3 + 4.5 e.u) + e.F / (2 rho cs^2) + neq (e e - cs^2 I) : B,
        // times kScale for 16-bit storage (which stores g / w_i) or w_i for FP32
        const R sc = S::lowp ? R(S::kScale) : R(1);
        const R P0 = (ps - R(1.5) * uu) * sc, A = R(0.5) * finv * sc, Nq = neq * sc;
        const R c3 = R(3) * sc, c45 = R(4.5) * sc;
        const R ct = trB * (R(1) / R(3));
        const R Bxy2 = R(2) * Bxy, Bxz2 = R(2) * Bxz, Byz2 = R(2) * Byz;
#pragma unroll
        for (int i = 0; i < QH; ++i) {
            const int ex = ev<QH>(i, 0), ey = ev<QH>(i, 1), ez = ev<QH>(i, 2);
            const R eu = R(ex) * ux + R(ey) * uy + R(ez) * uz;
            const R eF = R(ex) * F[0] + R(ey) * F[1] + R(ez) * F[2];
            const R eBe = R(ex * ex) * Bxx + R(ey * ey) * Byy + R(ez * ez) * Bzz + R(ex * ey) * Bxy2 +
                          R(ex * ez) * Bxz2 + R(ey * ez) * Byz2 - ct;
            const R sv = P0 + eu * (c3 + c45 * eu) + eF * A + eBe * Nq;
            if constexpr (S::lowp) io.store(i, S::raw_st(sv));
            else io.store(i, S::st(sv * wgt<QH, R>(i)));
        }
    } else {
#pragma unroll
        for (int i = 0; i < QH; ++i) {
            const int ex = ev<QH>(i, 0), ey = ev<QH>(i, 1), ez = ev<QH>(i, 2);
            const R w = wgt<QH, R>(i);
            const R geq = geq_i<S::QH, R>(i, ps, ux, uy, uz, uu);
            const R eF = R(ex) * F[0] + R(ey) * F[1] + R(ez) * F[2];
            // (e e - cs^2 I) : B
            const R eBe = R(ex * ex) * Bxx + R(ey * ey) * Byy + R(ez * ez) * Bzz +
                          R(2 * ex * ey) * Bxy + R(2 * ex * ez) * Bxz + R(2 * ey * ez) * Byz - c2 * trB;
            const R gs = geq + R(0.5) * w * eF * finv + neq * w * eBe;
            io.store(i, enc_g<S>(gs, i));
        }
    }
}

template <class S>
__global__ __launch_bounds__(kBlock) void k_hydro(const SweepArgs<S> a)
{
    const int c = xcd_block() * kBlock + threadIdx.x;
    if (c >= a.g.ncells) return;
    int x, y, z;
    Nbr n;
    if (!decode(a.g, c, x, y, z, n)) return;
    hydro_cell<S>(a, c, n, PhiG<typename S::real>{a.phi_in, c, &n}, IOGlobal<S, S::QH>{a.src, a.dst, c, &n, &a.g});
}

// ---- z-marching sweeps with the phase field staged in LDS ----------------------
// A block owns a kTX x kTY tile of (x, y) and walks zc consecutive planes.
// It keeps the phase field of planes z-1, z, z+1 over the tile plus a
// one-cell halo in a rotating set of three LDS buffers, so each plane of phi
// is read from memory once per tile (halo included) instead of once per
// neighbouring plane.  Wall rows are filled with their mirror (the adjacent
// fluid row), which is what the stencils read there.
struct ZTiles {
    int tx, ty, tz;  // tiles along x, y and z-chunks along z
    int zc;          // planes per z-chunk
};

__device__ inline int wrap_i(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ inline int mod_i(int v, int n) { return ((v % n) + n) % n; }

template <class R>
__device__ inline void load_plane(R *dst, const R *__restrict__ phi, const Grid &g, int x0, int y0, int z)
{
    const int zz = wrap_i(z, g.nz);
    for (int i = threadIdx.x; i < kLX * kLY; i += kBlock) {
        const int hx = i % kLX, hy = i / kLX;
        const int gx = mod_i(x0 - 1 + hx, g.nx);
        int gy = y0 - 1 + hy;
        if (g.walls) {
            gy = gy < 1 ? 1 : (gy > g.ny - 2 ? g.ny - 2 : gy);
        } else {
            gy = mod_i(gy, g.ny);
        }
        dst[i] = phi[gx + (int64_t)g.nx * (gy + (int64_t)g.ny * zz)];
    }
}

__device__ inline bool zm_cell(const Grid &g, const ZTiles &zt, int &x0, int &y0, int &z0, int &z1, int &x, int &y)
{
    int b = xcd_block();
    const int bx = b % zt.tx;
    b /= zt.tx;
    const int by = b % zt.ty;
    const int bz = b / zt.ty;
    x0 = bx * kTX;
    y0 = by * kTY;
    z0 = bz * zt.zc;
    z1 = z0 + zt.zc < g.nz ? z0 + zt.zc : g.nz;
    x = x0 + (int)(threadIdx.x % kTX);
    y = y0 + (int)(threadIdx.x / kTX);
    return x < g.nx && y < g.ny && !(g.walls && (y == 0 || y == g.ny - 1));
}

__device__ inline Nbr zm_nbr(const Grid &g, int x, int y, int z)
{
    Nbr n;
    const int nxy = g.nx * g.ny;
    n.xm = (x == 0) ? g.nx - 1 : -1;
    n.xp = (x == g.nx - 1) ? -(g.nx - 1) : 1;
    if (g.walls) {
        n.ym = -g.nx;
        n.yp = g.nx;
        n.wm = (y == 1);
        n.wp = (y == g.ny - 2);
    } else {
        n.ym = (y == 0) ? (g.ny - 1) * g.nx : -g.nx;
        n.yp = (y == g.ny - 1) ? -(g.ny - 1) * g.nx : g.nx;
        n.wm = n.wp = false;
    }
    n.zm = (z == 0) ? (g.nz - 1) * nxy : -nxy;
    n.zp = (z == g.nz - 1) ? -(g.nz - 1) * nxy : nxy;
    return n;
}

// PHASE: the phase sweep (stencil on phi_in, the previous field), else the
// hydrodynamic sweep (stencil on phi_in, the new field).
template <class S, bool PHASE>
__global__ __launch_bounds__(kBlock) void k_sweep_zm(const SweepArgs<S> a, const ZTiles zt)
{
    using R = typename S::real;
    __shared__ R buf[3][kLX * kLY];
    int x0, y0, z0, z1, x, y;
    const bool active = zm_cell(a.g, zt, x0, y0, z0, z1, x, y);
    const int o = (int)(threadIdx.x / kTX + 1) * kLX + (int)(threadIdx.x % kTX) + 1;
    load_plane(buf[0], a.phi_in, a.g, x0, y0, z0 - 1);
    load_plane(buf[1], a.phi_in, a.g, x0, y0, z0);
    int sm = 0, sc = 1, sp = 2;
    for (int z = z0; z < z1; ++z) {
        load_plane(buf[sp], a.phi_in, a.g, x0, y0, z + 1);
        __syncthreads();
        if (active) {
            const int c = x + a.g.nx * (y + a.g.ny * z);
            const Nbr n = zm_nbr(a.g, x, y, z);
            const PhiL<R> pl{{buf[sm], buf[sc], buf[sp]}, o};
            if constexpr (PHASE) phase_cell<S>(a, c, n, pl, IOGlobal<S, S::QP>{a.src, a.dst, c, &n, &a.g});
            else hydro_cell<S>(a, c, n, pl, IOGlobal<S, S::QH>{a.src, a.dst, c, &n, &a.g});
        }
        __syncthreads();
        const int t = sm;
        sm = sc;
        sc = sp;
        sp = t;
    }
}

// ---- paired sweeps for 16-bit storage ---------------------------------------
// One thread per pair of cells (x, y, z) and (x, y, z + nz/2) (nz even): the
// pair's 15 or 27 populations arrive as 32-bit words from the upstream pair
// in the half domain, so every load and store is 4 bytes instead of 2.
// Where the z pull wraps across the half domain (z = 0 pulling from below,
// z = nz/2 - 1 pulling from above) the upstream word holds the two cells the
// other way round and its halves are swapped.  Each cell then runs the same
// per-cell body as the one-cell-per-thread sweeps.
template <class S, bool PHASE>
__global__ __launch_bounds__(kBlock) void k_sweep_pair(const SweepArgs<S> a)
{
    static_assert(S::paired, "paired sweeps need 16-bit storage");
    constexpr int Q = PHASE ? S::QP : S::QH;
    using pdf_t = typename S::pdf_t;
    using R = typename S::real;
    const Grid &g = a.g;
    const int p = xcd_block() * kBlock + threadIdx.x;
    if (p >= g.half) return;
    const int t = (int)g.dnx.div((uint32_t)p);
    const int x = p - t * g.nx;
    const int z2 = (int)g.dny.div((uint32_t)t);
    const int y = t - z2 * g.ny;
    if (g.walls && (y == 0 || y == g.ny - 1)) return;
    const int nz2 = g.nz / 2, nxy = g.nx * g.ny;
    const int xm = (x == 0) ? g.nx - 1 : -1, xp = (x == g.nx - 1) ? -(g.nx - 1) : 1;
    int ym, yp;
    bool wm = false, wp = false;
    if (g.walls) {
        ym = -g.nx;
        yp = g.nx;
        wm = (y == 1);
        wp = (y == g.ny - 2);
    } else {
        ym = (y == 0) ? (g.ny - 1) * g.nx : -g.nx;
        yp = (y == g.ny - 1) ? -(g.ny - 1) * g.nx : g.nx;
    }
    const int zm = (z2 == 0) ? (nz2 - 1) * nxy : -nxy, zp = (z2 == nz2 - 1) ? -(nz2 - 1) * nxy : nxy;
    const uint32_t *__restrict__ W = reinterpret_cast<const uint32_t *>(a.src);
    uint32_t *__restrict__ Wd = reinterpret_cast<uint32_t *>(a.dst);
    pdf_t in0[Q], in1[Q], out0[Q], out1[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ex = ev<Q>(i, 0), ey = ev<Q>(i, 1), ez = ev<Q>(i, 2);
        const bool bb = (ey > 0 && wm) || (ey < 0 && wp);
        int64_t w;
        bool sw = false;
        if (bb) {
            w = pidx<Q>(opp(i), p);
        } else {
            const int off = (ex > 0 ? xm : ex < 0 ? xp : 0) + (ey > 0 ? ym : ey < 0 ? yp : 0) +
                            (ez > 0 ? zm : ez < 0 ? zp : 0);
            w = pidx<Q>(i, p + off);
            sw = (z2 == 0 && ez > 0) || (z2 == nz2 - 1 && ez < 0);
        }
        uint32_t v = ld_stream(W + w);
        if (sw) v = (v >> 16) | (v << 16);
        in0[i] = __builtin_bit_cast(pdf_t, (uint16_t)(v & 0xffffu));
        in1[i] = __builtin_bit_cast(pdf_t, (uint16_t)(v >> 16));
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = p + h * g.half;
        const Nbr n = zm_nbr(g, x, y, z2 + h * nz2);
        const PhiG<R> ph{a.phi_in, c, &n};
        const IORegs<S, Q> io{h ? in1 : in0, h ? out1 : out0};
        if constexpr (PHASE) phase_cell<S>(a, c, n, ph, io);
        else hydro_cell<S>(a, c, n, ph, io);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const uint32_t v = (uint32_t)__builtin_bit_cast(uint16_t, out0[i]) |
                           ((uint32_t)__builtin_bit_cast(uint16_t, out1[i]) << 16);
        st_stream(Wd + pidx<Q>(i, p), v);
    }
}

// ---- launch of one sweep ------------------------------------------------------
// The default pair (D3Q15 SRT phase field, D3Q27 hydrodynamics) has every
// sweep variant; the other velocity sets run the one-cell-per-thread sweeps.
template <class S>
constexpr bool is_default_lattice()
{
    return S::QP == 15 && S::QH == 27 && !S::phase_mrt;
}

// The sweeps for FP32 arithmetic (FP32 and 16-bit storage) are instantiated in
// their own translation unit, compiled with contraction of a*b+c into fused
// multiply-adds; the FP64 sweeps are instantiated with the rest of the
// library, without contraction.
struct SweepLaunch {
    int mode;    // 0: one cell per thread, 1: z-marching with LDS, 2: paired 16-bit
    int blocks;  // grid size
    ZTiles zt;   // tiling of mode 1
};

// The hydrodynamic sweep of step n and the phase-field sweep of step n + 1 on
// the same cell.  Step n + 1's phase sweep reads the h populations and the
// phase field that step n's phase sweep wrote (complete before this launch)
// and u at the cell only, which the hydrodynamic body has just computed and
// hands over in registers; the two bodies read the same phase field (the
// hydrodynamic one as the new field, the phase one as the previous field of
// its gradient) and touch disjoint buffers otherwise.  Same arithmetic as the
// two separate sweeps, one pass over the cells instead of two.
template <class S>
__global__ __launch_bounds__(kBlock) void k_fused(const SweepArgs<S> ah, const SweepArgs<S> ap)
{
    using R = typename S::real;
    const int c = xcd_block() * kBlock + threadIdx.x;
    if (c >= ah.g.ncells) return;
    int x, y, z;
    Nbr n;
    if (!decode(ah.g, c, x, y, z, n)) return;
    R un[3];
    hydro_cell<S, PhiG<R>, IOGlobal<S, S::QH>, true>(ah, c, n, PhiG<R>{ah.phi_in, c, &n},
                                                     IOGlobal<S, S::QH>{ah.src, ah.dst, c, &n, &ah.g}, un);
    phase_cell<S, PhiG<R>, IOGlobal<S, S::QP>, true>(ap, c, n, PhiG<R>{ap.phi_in, c, &n},
                                                     IOGlobal<S, S::QP>{ap.src, ap.dst, c, &n, &ap.g}, un);
}

template <class S>
void launch_fused(const SweepArgs<S> &ah, const SweepArgs<S> &ap, const SweepLaunch &L, hipStream_t stream)
{
    hipLaunchKernelGGL((k_fused<S>), dim3(L.blocks), dim3(kBlock), 0, stream, ah, ap);
}

template <class S, bool PHASE>
void launch_sweep(const SweepArgs<S> &a, const SweepLaunch &L, hipStream_t stream)
{
    if constexpr (S::paired) {
        if (L.mode == 2) {
            hipLaunchKernelGGL((k_sweep_pair<S, PHASE>), dim3(L.blocks), dim3(kBlock), 0, stream, a);
            return;
        }
    }
    if constexpr (is_default_lattice<S>()) {
        if (L.mode == 1) {
            hipLaunchKernelGGL((k_sweep_zm<S, PHASE>), dim3(L.blocks), dim3(kBlock), 0, stream, a, L.zt);
            return;
        }
    }
    if constexpr (PHASE) {
        hipLaunchKernelGGL((k_phase<S>), dim3(L.blocks), dim3(kBlock), 0, stream, a);
    } else {
        hipLaunchKernelGGL((k_hydro<S>), dim3(L.blocks), dim3(kBlock), 0, stream, a);
    }
}

// ---- the straightforward algorithm (Alg. naiveAlgorithm, Sec. 4.2) ----------
// Six passes per step instead of two sweeps: stream h, update phi, stream g,
// update u, collide h, collide g -- the order of the algorithm's loop, cut
// where the fused step's state sits (populations post-collision at the
// cell), so both share the initial state and the getters.  Each population
// set is read three times per step (stream, update or collide, and the
// collision of the new time), as the algorithm is written.  Time-consistent
// reading: the collisions take phi, its gradient, theta and u of the new
// time; the velocity update keeps the stored velocity inside the viscous
// force, as the fused step does; the collision of g recomputes the force
// with the updated velocity.  FP64 and FP32 storage.  The buffers: a = the
// current populations (post-collision), b = the other copy; after a step the
// state is in b.
template <class S, int Q>
struct IOCell {
    typename S::pdf_t *__restrict__ buf;  // read and written at the cell (in place)
    int c;
    const Grid *g;
    __device__ typename S::pdf_t load(int i) const { return buf[pdf_index<S, Q>(i, c, *g)]; }
    __device__ void store(int i, typename S::pdf_t v) const { st_stream(buf + pdf_index<S, Q>(i, c, *g), v); }
};

// dst(c) = src pulled from c - e_i (bounce-back at a wall), for every direction
template <class S, int Q>
__global__ __launch_bounds__(kBlock) void k_naive_stream(const typename S::pdf_t *__restrict__ src,
                                                         typename S::pdf_t *__restrict__ dst, const Grid g)
{
    const int c = xcd_block() * kBlock + threadIdx.x;
    if (c >= g.ncells) return;
    int x, y, z;
    Nbr n;
    if (!decode(g, c, x, y, z, n)) return;
#pragma unroll
    for (int i = 0; i < Q; ++i) st_stream(dst + pdf_index<S, Q>(i, c, g), ld_stream(src + pull_idx<S, Q>(i, c, n, g)));
}

// phi = sum of the streamed h at the cell (eq. updatePhaseField), summed in
// FP64 as the phase sweep sums it
template <class S>
__global__ __launch_bounds__(kBlock) void k_naive_phi(const typename S::pdf_t *__restrict__ h,
                                                      typename S::real *__restrict__ phi, const Grid g)
{
    const int c = xcd_block() * kBlock + threadIdx.x;
    if (c >= g.ncells) return;
    int x, y, z;
    Nbr n;
    if (!decode(g, c, x, y, z, n)) return;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < S::QP; ++i) {
        if constexpr (std::is_same<typename S::real, double>::value) acc += dec_h<S>(h[pdf_index<S, S::QP>(i, c, g)], 0.0, i);
        else acc += dec_h64<S>(h[pdf_index<S, S::QP>(i, c, g)], 0.f, i);
    }
    st_field(phi + c, typename S::real(acc));
}

// velocity update from the streamed g (a.dst) and the new phi (a.phi_in)
template <class S>
__global__ __launch_bounds__(kBlock) void k_naive_update_u(const SweepArgs<S> a)
{
    using R = typename S::real;
    const int c = xcd_block() * kBlock + threadIdx.x;
    if (c >= a.g.ncells) return;
    int x, y, z;
    Nbr n;
    if (!decode(a.g, c, x, y, z, n)) return;
    hydro_cell<S, PhiG<R>, IOCell<S, S::QH>, false, kHydroUpdateU>(a, c, n, PhiG<R>{a.phi_in, c, &n},
                                                                    IOCell<S, S::QH>{a.dst, c, &a.g});
}

// collision of the streamed h (a.dst, in place) with the new phi's stencil
template <class S>
__global__ __launch_bounds__(kBlock) void k_naive_collide_h(const SweepArgs<S> a)
{
    using R = typename S::real;
    const int c = xcd_block() * kBlock + threadIdx.x;
    if (c >= a.g.ncells) return;
    int x, y, z;
    Nbr n;
    if (!decode(a.g, c, x, y, z, n)) return;
    phase_cell<S, PhiG<R>, IOCell<S, S::QP>, false, false>(a, c, n, PhiG<R>{a.phi_in, c, &n},
                                                           IOCell<S, S::QP>{a.dst, c, &a.g});
}

// collision of the streamed g (a.dst, in place) with the updated u
template <class S>
__global__ __launch_bounds__(kBlock) void k_naive_collide_g(const SweepArgs<S> a)
{
    using R = typename S::real;
    const int c = xcd_block() * kBlock + threadIdx.x;
    if (c >= a.g.ncells) return;
    int x, y, z;
    Nbr n;
    if (!decode(a.g, c, x, y, z, n)) return;
    hydro_cell<S, PhiG<R>, IOCell<S, S::QH>, false, kHydroCollide>(a, c, n, PhiG<R>{a.phi_in, c, &n},
                                                                    IOCell<S, S::QH>{a.dst, c, &a.g});
}

// One step of the straightforward algorithm: H[a] -> H[b], G[a] -> G[b],
// phi[a] -> phi[b].  ph: h (a.src H[a], a.dst H[b]); gh: g (G[a], G[b]);
// both with phi_in = phi[b] (the new phase field) and phi_out = phi[b].
template <class S>
void launch_naive_step(const SweepArgs<S> &ph, const SweepArgs<S> &gh, int blocks, hipStream_t stream)
{
    hipLaunchKernelGGL((k_naive_stream<S, S::QP>), dim3(blocks), dim3(kBlock), 0, stream, ph.src, ph.dst, ph.g);
    hipLaunchKernelGGL((k_naive_phi<S>), dim3(blocks), dim3(kBlock), 0, stream, ph.dst, ph.phi_out, ph.g);
    hipLaunchKernelGGL((k_naive_stream<S, S::QH>), dim3(blocks), dim3(kBlock), 0, stream, gh.src, gh.dst, gh.g);
    hipLaunchKernelGGL((k_naive_update_u<S>), dim3(blocks), dim3(kBlock), 0, stream, gh);
    hipLaunchKernelGGL((k_naive_collide_h<S>), dim3(blocks), dim3(kBlock), 0, stream, ph);
    hipLaunchKernelGGL((k_naive_collide_g<S>), dim3(blocks), dim3(kBlock), 0, stream, gh);
}

// The FP32 storage types with other velocity sets (see Lattice).
using StoreF32_15_27_mrt = Lattice<StoreF32, 15, 27, true>;
using StoreF32_19_19 = Lattice<StoreF32, 19, 19, false>;
using StoreF32_19_19_mrt = Lattice<StoreF32, 19, 19, true>;
using StoreF32_27_27 = Lattice<StoreF32, 27, 27, false>;
using StoreF32_15_15 = Lattice<StoreF32, 15, 15, false>;
#define LBM_FP32_LATTICES(X) X(StoreF32_15_27_mrt) X(StoreF32_19_19) X(StoreF32_19_19_mrt) X(StoreF32_27_27) X(StoreF32_15_15)

#define LBM_FP32_SWEEPS(X)                                                                          \
    X(StoreF32, true) X(StoreF32, false) X(StoreF16S, true) X(StoreF16S, false) X(StoreBF16S, true) \
    X(StoreBF16S, false) X(StoreF32_15_27_mrt, true) X(StoreF32_15_27_mrt, false) X(StoreF32_19_19, true)    \
    X(StoreF32_19_19, false) X(StoreF32_19_19_mrt, true) X(StoreF32_19_19_mrt, false) X(StoreF32_27_27, true) \
    X(StoreF32_27_27, false) X(StoreF32_15_15, true) X(StoreF32_15_15, false)

// ---- initial / equilibrium state from (phi, u, p*) ---------------------------
// Writes the phase-field PDFs (post-collision, stored as is), the canonical
// pre-collision hydrodynamic PDFs into Gc (blocked layout; turned into the
// stored post-collision form by k_unpull), phi and u.
template <class S, class In>
__global__ __launch_bounds__(kBlock) void k_equilibrium(typename S::pdf_t *__restrict__ H,
                                                        typename S::pdf_t *__restrict__ Gc,
                                                        typename S::real *__restrict__ phiA,
                                                        typename S::real *__restrict__ u,
                                                        const In *__restrict__ phi_in,
                                                        const In *__restrict__ u_in,
                                                        const In *__restrict__ p_in, int p_is_pressure,
                                                        Grid g, Phys<typename S::real> ph)
{
    using R = typename S::real;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.ncells) return;
    const int y = (c / g.nx) % g.ny;
    const int64_t N = g.ncells;
    const bool wall = g.walls && (y == 0 || y == g.ny - 1);
    R phi = wall ? R(0) : R(phi_in[c]);
    R ux = wall ? R(0) : R(u_in[c]), uy = wall ? R(0) : R(u_in[N + c]), uz = wall ? R(0) : R(u_in[2 * N + c]);
    R ps = wall ? R(0) : R(p_in[c]);
    if (p_is_pressure && !wall) {
        const R rho = density_of(ph, phi);
        ps = ps / (rho * cs2<R>());
    }
    const R uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < S::QP; ++i) {
        const R h = wall ? R(0) : phi * gamma_i<S::QP, R>(i, ux, uy, uz, uu);
        H[pdf_index<S, S::QP>(i, c, g)] = enc_h<S>(h, phi, i);
    }
#pragma unroll
    for (int i = 0; i < S::QH; ++i) {
        const R ge = wall ? R(0) : geq_i<S::QH, R>(i, ps, ux, uy, uz, uu);
        Gc[pdf_index<S, S::QH>(i, c, g)] = enc_g<S>(ge, i);
    }
    phiA[c] = phi;
    u[c] = ux;
    u[g.fplane + c] = uy;
    u[2 * g.fplane + c] = uz;
}

// Stored post-collision G from canonical pre-collision Gc: the population of
// direction j stored at cell y is the one that arrives at y + e_j (or, if
// y + e_j is a wall, the reversed one arriving back at y).  Exact inverse of
// the pull of the sweeps.  Wall cells are left untouched.
template <class S>
__global__ __launch_bounds__(kBlock) void k_unpull(const typename S::pdf_t *__restrict__ Gc,
                                                     typename S::pdf_t *__restrict__ G, Grid g)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.ncells) return;
    int x, y, z;
    Nbr n;
    if (!decode(g, c, x, y, z, n)) return;
#pragma unroll
    for (int j = 0; j < S::QH; ++j) {
        const int dx = ev<S::QH>(j, 0), dy = ev<S::QH>(j, 1), dz = ev<S::QH>(j, 2);
        const bool bb = (dy > 0 && n.wp) || (dy < 0 && n.wm);  // y + e_j is a wall row
        const int64_t from = bb ? pdf_index<S, S::QH>(opp(j), c, g) : pdf_index<S, S::QH>(j, c + n.off(dx, dy, dz), g);
        G[pdf_index<S, S::QH>(j, c, g)] = Gc[from];
    }
}

// Canonical FP64 planes from storage: H as stored, G pulled (pre-collision).
template <class S>
__global__ __launch_bounds__(kBlock) void k_get_pdfs(const typename S::pdf_t *__restrict__ H,
                                                     const typename S::pdf_t *__restrict__ G,
                                                     const typename S::real *__restrict__ phiA,
                                                     double *__restrict__ Ho, double *__restrict__ Go,
                                                     Grid g, Phys<typename S::real> ph)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.ncells) return;
    const int64_t N = g.ncells;
    int x, y, z;
    Nbr n;
    const bool fluid = decode(g, c, x, y, z, n);
    if (Ho)
#pragma unroll
        for (int i = 0; i < S::QP; ++i)
            Ho[i * N + c] = fluid ? (double)dec_h<S>(H[pdf_index<S, S::QP>(i, c, g)], phiA[c], i) : 0.0;
    if (Go)
#pragma unroll
        for (int i = 0; i < S::QH; ++i)
            Go[i * N + c] = fluid ? (double)dec_g<S>(G[pull_idx<S, S::QH>(i, c, n, g)], i) : 0.0;
}

// Storage from canonical FP64 planes: H stored directly, G (pre-collision)
// written to Gc in storage format, to be turned into the stored form by
// k_unpull.
template <class S>
__global__ __launch_bounds__(kBlock) void k_set_pdfs(typename S::pdf_t *__restrict__ H,
                                                     typename S::pdf_t *__restrict__ Gc,
                                                     typename S::real *__restrict__ phiA,
                                                     typename S::real *__restrict__ u,
                                                     const double *__restrict__ Hi, const double *__restrict__ Gi,
                                                     const double *__restrict__ phi_i,
                                                     const double *__restrict__ u_i, Grid g,
                                                     Phys<typename S::real> ph)
{
    using R = typename S::real;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.ncells) return;
    const int y = (c / g.nx) % g.ny;
    const bool wall = g.walls && (y == 0 || y == g.ny - 1);
    const int64_t N = g.ncells;
#pragma unroll
    for (int i = 0; i < S::QP; ++i) {
        H[pdf_index<S, S::QP>(i, c, g)] = enc_h<S>(wall ? R(0) : R(Hi[i * N + c]), wall ? R(0) : R(phi_i[c]), i);
    }
#pragma unroll
    for (int i = 0; i < S::QH; ++i) Gc[pdf_index<S, S::QH>(i, c, g)] = enc_g<S>(wall ? R(0) : R(Gi[i * N + c]), i);
    phiA[c] = wall ? R(0) : R(phi_i[c]);
    for (int k = 0; k < 3; ++k) u[k * g.fplane + c] = wall ? R(0) : R(u_i[k * N + c]);
}

// Moving the state to new macroscopic fields (phi', u', p') while keeping
// every population's non-equilibrium part: the populations gain the change
// of their equilibria, h_i += phi' Gamma_i(u') - phi Gamma_i(u) and
// g_i += g^eq_i(p*', u') - g^eq_i(p*, u), with phi, u the stored fields and
// p* = sum_i g_i.  First the canonical pre-collision G (pulled, as in the
// hydrodynamic sweep) with its increment into Gc, which k_unpull turns
// back into the stored form; it reads the old u, so it runs before
// k_shift_eq_h.  Wall cells are left as they are.
template <class S, class In>
__global__ __launch_bounds__(kBlock) void k_shift_eq_g(const typename S::pdf_t *__restrict__ G,
                                                       typename S::pdf_t *__restrict__ Gc,
                                                       const typename S::real *__restrict__ u,
                                                       const In *__restrict__ phi_in, const In *__restrict__ u_in,
                                                       const In *__restrict__ p_in, Grid g,
                                                       Phys<typename S::real> ph)
{
    using R = typename S::real;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.ncells) return;
    int x, y, z;
    Nbr n;
    if (!decode(g, c, x, y, z, n)) return;
    const int64_t N = g.ncells;
    R gc[S::QH], ps = R(0);
#pragma unroll
    for (int i = 0; i < S::QH; ++i) {
        gc[i] = dec_g<S>(G[pull_idx<S, S::QH>(i, c, n, g)], i);
        ps += gc[i];
    }
    const R ux = u[c], uy = u[g.fplane + c], uz = u[2 * g.fplane + c];
    const R uu = ux * ux + uy * uy + uz * uz;
    const R vx = R(u_in[c]), vy = R(u_in[N + c]), vz = R(u_in[2 * N + c]);
    const R vv = vx * vx + vy * vy + vz * vz;
    const R qs = R(p_in[c]) / (density_of(ph, R(phi_in[c])) * cs2<R>());
#pragma unroll
    for (int i = 0; i < S::QH; ++i) {
        const R gn = gc[i] + (geq_i<S::QH, R>(i, qs, vx, vy, vz, vv) - geq_i<S::QH, R>(i, ps, ux, uy, uz, uu));
        Gc[pdf_index<S, S::QH>(i, c, g)] = enc_g<S>(gn, i);
    }
}

// Second part of the move: h (post-collision, stored at the cell) gains the
// change of phi Gamma(u); then phi_A and u take the new values.
template <class S, class In>
__global__ __launch_bounds__(kBlock) void k_shift_eq_h(typename S::pdf_t *__restrict__ H,
                                                       typename S::real *__restrict__ phiA,
                                                       typename S::real *__restrict__ u,
                                                       const In *__restrict__ phi_in, const In *__restrict__ u_in,
                                                       Grid g)
{
    using R = typename S::real;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.ncells) return;
    const int y = (c / g.nx) % g.ny;
    if (g.walls && (y == 0 || y == g.ny - 1)) return;
    const int64_t N = g.ncells;
    const R phi = phiA[c];
    const R ux = u[c], uy = u[g.fplane + c], uz = u[2 * g.fplane + c];
    const R uu = ux * ux + uy * uy + uz * uz;
    const R phn = R(phi_in[c]);
    const R vx = R(u_in[c]), vy = R(u_in[N + c]), vz = R(u_in[2 * N + c]);
    const R vv = vx * vx + vy * vy + vz * vz;
#pragma unroll
    for (int i = 0; i < S::QP; ++i) {
        const int64_t k = pdf_index<S, S::QP>(i, c, g);
        const R h = dec_h<S>(H[k], phi, i) +
                    (phn * gamma_i<S::QP, R>(i, vx, vy, vz, vv) - phi * gamma_i<S::QP, R>(i, ux, uy, uz, uu));
        H[k] = enc_h<S>(h, phn, i);
    }
    phiA[c] = phn;
    u[c] = vx;
    u[g.fplane + c] = vy;
    u[2 * g.fplane + c] = vz;
}

template <class S, class Out>
__global__ __launch_bounds__(kBlock) void k_get_macro(const typename S::pdf_t *__restrict__ G,
                                                      const typename S::real *__restrict__ phiA,
                                                      const typename S::real *__restrict__ u,
                                                      Out *__restrict__ phi_o, Out *__restrict__ u_o,
                                                      Out *__restrict__ p_o, Grid g,
                                                      Phys<typename S::real> ph)
{
    using R = typename S::real;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.ncells) return;
    int x, y, z;
    Nbr n;
    const bool fluid = decode(g, c, x, y, z, n);
    const int64_t N = g.ncells;
    if (phi_o) phi_o[c] = fluid ? Out(phiA[c]) : Out(0);
    if (u_o)
        for (int k = 0; k < 3; ++k) u_o[k * N + c] = fluid ? Out(u[k * g.fplane + c]) : Out(0);
    if (p_o) {
        R ps = R(0);
        if (fluid)
#pragma unroll
            for (int i = 0; i < S::QH; ++i) ps += dec_g<S>(G[pull_idx<S, S::QH>(i, c, n, g)], i);
        const R rho = density_of(ph, phiA[c]);
        p_o[c] = fluid ? Out(ps * rho * cs2<R>()) : Out(0);
    }
}

// ---- deterministic FP64 reductions --------------------------------------------
// Pass 1: a fixed grid of kRedBlocks blocks; thread t of block b visits
// cells b*kBlock + t + k*kRedBlocks*kBlock in order.  Each wavefront combines
// its 64 lanes with a butterfly of cross-lane exchanges (every lane ends with
// the same value), the wavefronts' results are combined in wave order, and
// the block writes its partials.  Pass 2: one block combines the block
// partials the same way.  Same result for every run on any device.
constexpr int kWaves = kBlock / 64;

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Leaves the block's totals in sh[0 .. kRedVals-1] (sh holds kRedVals*kWaves).
__device__ inline void block_reduce(double v[kRedVals], double *sh)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kRedVals; ++k) v[k] = (k == kRedVals - 1) ? wave_max(v[k]) : wave_sum(v[k]);
    if (lane == 0)
        for (int k = 0; k < kRedVals; ++k) sh[k * kWaves + w] = v[k];
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x < kRedVals) {
        const int k = threadIdx.x;
        r = sh[k * kWaves];
        for (int i = 1; i < kWaves; ++i) r = (k == kRedVals - 1) ? fmax(r, sh[k * kWaves + i]) : r + sh[k * kWaves + i];
    }
    __syncthreads();
    if (threadIdx.x < kRedVals) sh[threadIdx.x] = r;
    __syncthreads();
}

template <class S>
__global__ __launch_bounds__(kBlock) void k_reduce1(const typename S::real *__restrict__ phiA,
                                                    const typename S::real *__restrict__ u, Grid g,
                                                    Phys<typename S::real> ph, int mass_only,
                                                    double *__restrict__ partial)
{
    using R = typename S::real;
    __shared__ double sh[kRedVals * kWaves];
    double v[kRedVals];
    for (int k = 0; k < kRedVals; ++k) v[k] = 0.0;
    const double phiH = (double)ph.phi_H, phiL = (double)ph.phi_L, idp = (double)ph.inv_dphi;
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < g.ncells; c += kRedBlocks * kBlock) {
        int x, y, z;
        Nbr n;
        if (!decode(g, c, x, y, z, n)) continue;
        const double phi = (double)phiA[c];
        v[0] += phi;
        if (mass_only) continue;
        const double phc = phi < (double)ph.phi_lo ? (double)ph.phi_lo : (phi > (double)ph.phi_hi ? (double)ph.phi_hi : phi);
        const double rho = (double)ph.rho_L + (phc - phiL) * (double)ph.drho * idp;
        const double ux = u[c], uy = u[g.fplane + c], uz = u[2 * g.fplane + c];
        const double chi = (phiH - phi) * idp;
        R grad[3], lapu;
        stencil<27, R, false>(PhiG<R>{phiA, c, &n}, grad, lapu);
        const double gn = sqrt((double)grad[0] * grad[0] + (double)grad[1] * grad[1] + (double)grad[2] * grad[2]);
        v[1] += rho * ux;
        v[2] += rho * uy;
        v[3] += rho * uz;
        v[4] += chi;
        v[5] += chi * x;
        v[6] += chi * y;
        v[7] += chi * z;
        v[8] += chi * uy;
        v[9] += 4.0 * chi * (1.0 - chi);
        v[10] += gn * idp;
        v[11] = fmax(v[11], sqrt(ux * ux + uy * uy + uz * uz));
    }
    block_reduce(v, sh);
    if (threadIdx.x < kRedVals) partial[blockIdx.x * kRedVals + threadIdx.x] = sh[threadIdx.x];
}

#ifndef LBM_SWEEPS_ONLY  // non-template kernels: defined once, in the translation unit of the C ABI
__global__ __launch_bounds__(kBlock) void k_reduce2(const double *__restrict__ partial,
                                                    double *__restrict__ out)
{
    __shared__ double sh[kRedVals * kWaves];
    double v[kRedVals];
    for (int k = 0; k < kRedVals; ++k) v[k] = 0.0;
    for (int b = threadIdx.x; b < kRedBlocks; b += kBlock)
        for (int k = 0; k < kRedVals; ++k) {
            const double o = partial[b * kRedVals + k];
            v[k] = (k == kRedVals - 1) ? fmax(v[k], o) : v[k] + o;
        }
    block_reduce(v, sh);
    if (threadIdx.x < kRedVals) out[threadIdx.x] = sh[threadIdx.x];
}

// ---- fill with zeros (16-byte vectors); used instead of a runtime memset so
// the calls stay plain kernels --------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_zero(uint4 *__restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = make_uint4(0, 0, 0, 0);
}

// ---- STREAM copy a_i = b_i (16-byte vectors, one per thread, no loop: the
// fastest of the copy shapes measured on gfx950) -------------------------------
__global__ __launch_bounds__(kBlock) void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                 int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

#endif  // LBM_SWEEPS_ONLY

}  // namespace lbm
