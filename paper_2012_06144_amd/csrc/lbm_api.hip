// C ABI of the gfx950 coupled phase-field / hydrodynamic LBM solver
// (declarations and argument contracts in include/lbm.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>

#include "lbm.h"
#include "lbm_kernels.hpp"

// FP32-arithmetic sweeps live in lbm_sweeps_f32.hip (compiled with FMA contraction)
namespace lbm {
#define LBM_EXTERN_SWEEP(S, P) extern template void launch_sweep<S, P>(const SweepArgs<S> &, const SweepLaunch &, hipStream_t);
LBM_FP32_SWEEPS(LBM_EXTERN_SWEEP)
#undef LBM_EXTERN_SWEEP
extern template void launch_fused<StoreF32>(const SweepArgs<StoreF32> &, const SweepArgs<StoreF32> &,
                                            const SweepLaunch &, hipStream_t);
extern template void launch_naive_step<StoreF32>(const SweepArgs<StoreF32> &, const SweepArgs<StoreF32> &, int,
                                                 hipStream_t);
#define LBM_EXTERN_LATTICE(S)                                                                                  \
    extern template void launch_fused<S>(const SweepArgs<S> &, const SweepArgs<S> &, const SweepLaunch &, hipStream_t); \
    extern template void launch_naive_step<S>(const SweepArgs<S> &, const SweepArgs<S> &, int, hipStream_t);
LBM_FP32_LATTICES(LBM_EXTERN_LATTICE)
#undef LBM_EXTERN_LATTICE
}  // namespace lbm

using namespace lbm;

namespace {

thread_local char g_err[512] = "";

lbm_status fail(lbm_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(LBM_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                               \
    } while (0)

#define LAUNCH_CHECK()                                                                               \
    do {                                                                                             \
        hipError_t e_ = hipGetLastError();                                                           \
        if (e_ != hipSuccess)                                                                        \
            return fail(LBM_EHIP, "kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                                   \
    } while (0)

constexpr size_t kAlign = 256;
// Extra elements between the three velocity planes so that the streams of
// one cell do not start on the same HBM channel when nx*ny*nz is a large
// power of two.
constexpr int64_t kPlanePadElems = 512;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t pdf_bytes(int storage) { return storage == LBM_F64 ? 8 : storage == LBM_F32 ? 4 : 2; }
size_t real_bytes(int storage) { return storage == LBM_F64 ? 8 : 4; }

// Velocity sets and phase-field collision of a parameter set (0 = default).
int q_phase(const lbm_params *p) { return p->lattice_phase == 0 ? 15 : p->lattice_phase; }
int q_hydro(const lbm_params *p) { return p->lattice_hydro == 0 ? 27 : p->lattice_hydro; }

// The built lattice variants: 0 is (D3Q15, D3Q27, SRT), every storage; the
// others FP64 and FP32 only.  -1: not built.
int lattice_variant(const lbm_params *p)
{
    const int qp = q_phase(p), qh = q_hydro(p), mrt = p->phase_mrt;
    if (qp == 15 && qh == 27 && mrt == 0) return 0;
    if (p->storage != LBM_F64 && p->storage != LBM_F32) return -1;
    if (qp == 15 && qh == 27 && mrt == 1) return 1;
    if (qp == 19 && qh == 19 && mrt == 0) return 2;
    if (qp == 19 && qh == 19 && mrt == 1) return 3;
    if (qp == 27 && qh == 27 && mrt == 0) return 4;
    if (qp == 15 && qh == 15 && mrt == 0) return 5;
    return -1;
}

struct Layout {
    int64_t ncells, nblk, fplane;
    int64_t pdf_elems;  // elements per direction of a PDF buffer
    size_t off_H[2], off_G[2], off_phi[2], off_u, off_red, off_out, total;
};

lbm_status validate(const lbm_params *p)
{
    if (!p) return fail(LBM_EARG, "params is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBM_EARG, "grid dimensions must be >= 1");
    if (p->walls_y && p->ny < 3) return fail(LBM_EARG, "walls_y needs ny >= 3");
    const int64_t n = (int64_t)p->nx * p->ny * p->nz;
    if (n > (int64_t)0x7fffffff - 4096) return fail(LBM_ESIZE, "grid of %lld cells exceeds 2^31", (long long)n);
    if (p->storage < LBM_F64 || p->storage > LBM_BF16S) return fail(LBM_EARG, "unknown storage %d", p->storage);
    if (!(p->phi_H != p->phi_L)) return fail(LBM_EARG, "phi_H must differ from phi_L");
    if (!(p->xi > 0)) return fail(LBM_EARG, "xi must be > 0");
    if (!(p->mobility > 0)) return fail(LBM_EARG, "mobility must be > 0 (phase relaxation rate in (0,2))");
    if (!(p->tau_L > 0) || !(p->tau_H > 0))
        return fail(LBM_EARG, "tau_L and tau_H must be > 0 (relaxation rates in (0,2))");
    if (!(p->rho_L > 0) || !(p->rho_H > 0)) return fail(LBM_EARG, "densities must be > 0");
    if (!(p->sigma >= 0)) return fail(LBM_EARG, "sigma must be >= 0");
    if (!(p->normal_eps >= 0)) return fail(LBM_EARG, "normal_eps must be >= 0");
    if (p->density_literal != 0 && p->density_literal != 1) return fail(LBM_EARG, "density_literal must be 0 or 1");
    if (p->phase_mrt != 0 && p->phase_mrt != 1) return fail(LBM_EARG, "phase_mrt must be 0 or 1");
    if (lattice_variant(p) < 0)
        return fail(LBM_EARG, "lattice pair (D3Q%d, D3Q%d, %s) with storage %d is not built", q_phase(p), q_hydro(p),
                    p->phase_mrt ? "MRT" : "SRT", p->storage);
    return LBM_OK;
}

Layout layout(const lbm_params *p)
{
    Layout L{};
    L.ncells = (int64_t)p->nx * p->ny * p->nz;
    L.nblk = (L.ncells + kB - 1) / kB;  // blocked PDF layout, kB cells per block
    L.fplane = (int64_t)align_up((size_t)L.ncells, 512) + kPlanePadElems;
    if (pdf_bytes(p->storage) == 2) {
        // paired 16-bit storage: ceil(N/2) words of two cells, in blocks of kB words
        const int64_t half = (L.ncells + 1) / 2;
        L.pdf_elems = 2 * ((half + kB - 1) / kB) * kB;
    } else {
        L.pdf_elems = L.nblk * kB;
    }
    const size_t pb = pdf_bytes(p->storage), rb = real_bytes(p->storage);
    size_t off = 0;
    for (int k = 0; k < 2; ++k) {
        L.off_H[k] = off;
        off = align_up(off + (size_t)q_phase(p) * (size_t)L.pdf_elems * pb, kAlign);
    }
    for (int k = 0; k < 2; ++k) {
        L.off_G[k] = off;
        off = align_up(off + (size_t)q_hydro(p) * (size_t)L.pdf_elems * pb, kAlign);
    }
    for (int k = 0; k < 2; ++k) {
        L.off_phi[k] = off;
        off = align_up(off + (size_t)L.fplane * rb, kAlign);
    }
    L.off_u = off;
    off = align_up(off + 3 * (size_t)L.fplane * rb, kAlign);
    L.off_red = off;
    off = align_up(off + (size_t)kRedBlocks * kRedVals * sizeof(double), kAlign);
    L.off_out = off;
    off = align_up(off + 16 * sizeof(double), kAlign);
    L.total = off;
    return L;
}

template <class R>
Phys<R> make_phys(const lbm_params *p)
{
    const double CS2 = 1.0 / 3.0;
    Phys<R> ph{};
    ph.phi_L = (R)p->phi_L;
    ph.phi_H = (R)p->phi_H;
    ph.phi_0 = (R)(0.5 * (p->phi_L + p->phi_H));
    ph.inv_dphi = (R)(1.0 / (p->phi_H - p->phi_L));
    if (p->density_literal) {
        // no clamp: the interpolations of eq. density for every phi
        ph.phi_lo = -std::numeric_limits<R>::max();
        ph.phi_hi = std::numeric_limits<R>::max();
    } else {
        ph.phi_lo = (R)(p->phi_L < p->phi_H ? p->phi_L : p->phi_H);
        ph.phi_hi = (R)(p->phi_L < p->phi_H ? p->phi_H : p->phi_L);
    }
    ph.xi = (R)p->xi;
    ph.inv_xi = (R)(1.0 / p->xi);
    const double tau_phi = p->mobility / CS2;  // eq. mobility with dt = 1
    ph.omega_phi = (R)(1.0 / (tau_phi + 0.5));
    ph.rho_L = (R)p->rho_L;
    ph.drho = (R)(p->rho_H - p->rho_L);
    ph.tau_L = (R)p->tau_L;
    ph.dtau = (R)(p->tau_H - p->tau_L);
    ph.beta = (R)(12.0 * p->sigma / p->xi);
    ph.kappa = (R)(1.5 * p->sigma * p->xi);
    for (int k = 0; k < 3; ++k) ph.accel[k] = (R)p->body_accel[k];
    ph.rho_ref = (R)p->buoyancy_rho_ref;
    ph.normal_eps = (R)p->normal_eps;
    return ph;
}

}  // namespace

struct lbm_ctx {
    lbm_params p;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    Layout L;
    Grid g;
    int cur;  // index of the current source buffers (H, G, phi)
    bool initialized;
    int64_t steps;
    bool zmarch;  // sweeps march in z with phi staged in LDS
    bool pair16;  // 16-bit storage with even nz: one thread per pair of cells
    bool fuse;    // lbm_step runs the hydrodynamic sweep of one step with the phase sweep of the next
};

namespace {

template <class S>
struct Ops {
    using pdf_t = typename S::pdf_t;
    using R = typename S::real;

    static pdf_t *H(lbm_ctx *c, int k) { return (pdf_t *)(c->ws + c->L.off_H[k]); }
    static pdf_t *G(lbm_ctx *c, int k) { return (pdf_t *)(c->ws + c->L.off_G[k]); }
    static R *phi(lbm_ctx *c, int k) { return (R *)(c->ws + c->L.off_phi[k]); }
    static R *u(lbm_ctx *c) { return (R *)(c->ws + c->L.off_u); }
    static int blocks(lbm_ctx *c) { return (int)((c->g.ncells + kBlock - 1) / kBlock); }

    // Tiling of the z-marching sweeps: about kZmBlocks blocks, at most 64
    // planes per block.
    static ZTiles ztiles(lbm_ctx *c)
    {
        ZTiles t;
        t.tx = (c->g.nx + kTX - 1) / kTX;
        t.ty = (c->g.ny + kTY - 1) / kTY;
        const int64_t tiles = (int64_t)t.tx * t.ty;
        int64_t zc = tiles * c->g.nz / kZmBlocks;
        zc = zc < 1 ? 1 : (zc > 64 ? 64 : zc);
        t.zc = (int)zc;
        t.tz = (c->g.nz + t.zc - 1) / t.zc;
        return t;
    }

    // paired 16-bit sweeps: one thread per two cells (needs even nz)
    static bool paired(lbm_ctx *c) { return S::paired && c->pair16 && c->g.nz % 2 == 0; }

    static SweepLaunch sweep_launch(lbm_ctx *c)
    {
        SweepLaunch L{};
        if (paired(c)) {
            L.mode = 2;
            L.blocks = (c->g.half + kBlock - 1) / kBlock;
        } else if (is_default_lattice<S>() && c->zmarch) {
            L.mode = 1;
            L.zt = ztiles(c);
            L.blocks = L.zt.tx * L.zt.ty * L.zt.tz;
        } else {
            L.mode = 0;
            L.blocks = blocks(c);
        }
        return L;
    }

    static void launch_phase(lbm_ctx *c, const SweepArgs<S> &sp)
    {
        launch_sweep<S, true>(sp, sweep_launch(c), c->stream);
    }

    static void launch_hydro(lbm_ctx *c, const SweepArgs<S> &sh)
    {
        launch_sweep<S, false>(sh, sweep_launch(c), c->stream);
    }

    static lbm_status zero_all(lbm_ctx *c)
    {
        const int64_t n = (int64_t)(c->L.off_red / 16);  // off_red is 256-byte aligned
        hipLaunchKernelGGL(k_zero, dim3(4096), dim3(kBlock), 0, c->stream, (uint4 *)c->ws, n);
        LAUNCH_CHECK();
        return LBM_OK;
    }

    template <class In>
    static lbm_status equilibrium(lbm_ctx *c, const In *phi_in, const In *u_in, const In *p_in, int is_p)
    {
        lbm_status s = zero_all(c);
        if (s != LBM_OK) return s;
        c->cur = 0;
        hipLaunchKernelGGL((k_equilibrium<S, In>), dim3(blocks(c)), dim3(kBlock), 0, c->stream, H(c, 0),
                           G(c, 1), phi(c, 0), u(c), phi_in, u_in, p_in, is_p, c->g, make_phys<R>(&c->p));
        LAUNCH_CHECK();
        hipLaunchKernelGGL((k_unpull<S>), dim3(blocks(c)), dim3(kBlock), 0, c->stream, G(c, 1), G(c, 0), c->g);
        LAUNCH_CHECK();
        c->initialized = true;
        c->steps = 0;
        return LBM_OK;
    }

    template <class In>
    static lbm_status shift_equilibrium(lbm_ctx *c, const In *phi_in, const In *u_in, const In *p_in)
    {
        const int a = c->cur, b = 1 - c->cur;
        const Phys<R> ph = make_phys<R>(&c->p);
        hipLaunchKernelGGL((k_shift_eq_g<S, In>), dim3(blocks(c)), dim3(kBlock), 0, c->stream, G(c, a), G(c, b),
                           u(c), phi_in, u_in, p_in, c->g, ph);
        LAUNCH_CHECK();
        hipLaunchKernelGGL((k_unpull<S>), dim3(blocks(c)), dim3(kBlock), 0, c->stream, G(c, b), G(c, a), c->g);
        LAUNCH_CHECK();
        hipLaunchKernelGGL((k_shift_eq_h<S, In>), dim3(blocks(c)), dim3(kBlock), 0, c->stream, H(c, a), phi(c, a),
                           u(c), phi_in, u_in, c->g);
        LAUNCH_CHECK();
        return LBM_OK;
    }

    static lbm_status step(lbm_ctx *c, int n)
    {
        const Phys<R> ph = make_phys<R>(&c->p);
        if constexpr (!S::paired) {
            const SweepLaunch L = sweep_launch(c);
            if (c->fuse && n >= 2 && L.mode == 0) {
                // phase(0); then hydro(t - 1) fused with phase(t); then hydro(n - 1)
                int a = c->cur, b = 1 - c->cur;
                SweepArgs<S> sp{H(c, a), H(c, b), phi(c, a), phi(c, b), u(c), c->g, ph};
                launch_phase(c, sp);
                LAUNCH_CHECK();
                for (int t = 1; t < n; ++t) {
                    SweepArgs<S> sh{G(c, a), G(c, b), phi(c, b), nullptr, u(c), c->g, ph};
                    SweepArgs<S> sq{H(c, b), H(c, a), phi(c, b), phi(c, a), u(c), c->g, ph};
                    launch_fused<S>(sh, sq, L, c->stream);
                    LAUNCH_CHECK();
                    a = b;
                    b = 1 - b;
                    ++c->steps;
                }
                SweepArgs<S> sh{G(c, a), G(c, b), phi(c, b), nullptr, u(c), c->g, ph};
                launch_hydro(c, sh);
                LAUNCH_CHECK();
                c->cur = b;
                ++c->steps;
                return LBM_OK;
            }
        }
        for (int t = 0; t < n; ++t) {
            const int a = c->cur, b = 1 - c->cur;
            SweepArgs<S> sp{H(c, a), H(c, b), phi(c, a), phi(c, b), u(c), c->g, ph};
            launch_phase(c, sp);
            LAUNCH_CHECK();
            SweepArgs<S> sh{G(c, a), G(c, b), phi(c, b), nullptr, u(c), c->g, ph};
            launch_hydro(c, sh);
            LAUNCH_CHECK();
            c->cur = b;
            ++c->steps;
        }
        return LBM_OK;
    }

    // n steps of the straightforward algorithm (six passes per step)
    static lbm_status step_straightforward(lbm_ctx *c, int n)
    {
        if constexpr (S::lowp) {
            return fail(LBM_EARG, "the straightforward algorithm runs with FP64 or FP32 storage");
        } else {
            const Phys<R> ph = make_phys<R>(&c->p);
            for (int t = 0; t < n; ++t) {
                const int a = c->cur, b = 1 - c->cur;
                SweepArgs<S> sp{H(c, a), H(c, b), phi(c, b), phi(c, b), u(c), c->g, ph};
                SweepArgs<S> sg{G(c, a), G(c, b), phi(c, b), nullptr, u(c), c->g, ph};
                launch_naive_step<S>(sp, sg, blocks(c), c->stream);
                LAUNCH_CHECK();
                c->cur = b;
                ++c->steps;
            }
            return LBM_OK;
        }
    }

    static lbm_status step_timed(lbm_ctx *c, int n, double *phase_ms, double *hydro_ms)
    {
        const Phys<R> ph = make_phys<R>(&c->p);
        hipEvent_t ev[3];
        for (int k = 0; k < 3; ++k) HIP_TRY(hipEventCreate(&ev[k]));
        double tp = 0.0, th = 0.0;
        lbm_status st = LBM_OK;
        for (int t = 0; t < n && st == LBM_OK; ++t) {
            const int a = c->cur, b = 1 - c->cur;
            SweepArgs<S> sp{H(c, a), H(c, b), phi(c, a), phi(c, b), u(c), c->g, ph};
            SweepArgs<S> sh{G(c, a), G(c, b), phi(c, b), nullptr, u(c), c->g, ph};
            hipError_t e = hipEventRecord(ev[0], c->stream);
            if (e == hipSuccess) {
                launch_phase(c, sp);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
            if (e == hipSuccess) {
                launch_hydro(c, sh);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipEventRecord(ev[2], c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
            float m1 = 0.f, m2 = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&m1, ev[0], ev[1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&m2, ev[1], ev[2]);
            if (e != hipSuccess) {
                st = fail(LBM_EHIP, "timed step failed: %s", hipGetErrorString(e));
                break;
            }
            tp += m1;
            th += m2;
            c->cur = b;
            ++c->steps;
        }
        for (int k = 0; k < 3; ++k) (void)hipEventDestroy(ev[k]);
        if (st != LBM_OK) return st;
        *phase_ms = tp / n;
        *hydro_ms = th / n;
        return LBM_OK;
    }

    // n >= 2 steps as lbm_step runs them with fused sweeps, HIP events around
    // every fused launch; mean fused-kernel time in ms.
    static lbm_status step_timed_fused(lbm_ctx *c, int n, double *fused_ms)
    {
        if constexpr (S::paired) {
            return fail(LBM_EARG, "16-bit storage has no fused sweep kernel");
        } else {
            const SweepLaunch L = sweep_launch(c);
            if (L.mode != 0) return fail(LBM_EARG, "the fused sweep kernel needs the one-cell-per-thread sweeps");
            const Phys<R> ph = make_phys<R>(&c->p);
            hipEvent_t ev[2];
            for (int k = 0; k < 2; ++k) HIP_TRY(hipEventCreate(&ev[k]));
            int a = c->cur, b = 1 - c->cur;
            SweepArgs<S> sp{H(c, a), H(c, b), phi(c, a), phi(c, b), u(c), c->g, ph};
            launch_phase(c, sp);
            hipError_t e = hipGetLastError();
            double tf = 0.0;
            for (int t = 1; t < n && e == hipSuccess; ++t) {
                SweepArgs<S> sh{G(c, a), G(c, b), phi(c, b), nullptr, u(c), c->g, ph};
                SweepArgs<S> sq{H(c, b), H(c, a), phi(c, b), phi(c, a), u(c), c->g, ph};
                e = hipEventRecord(ev[0], c->stream);
                if (e == hipSuccess) {
                    launch_fused<S>(sh, sq, L, c->stream);
                    e = hipGetLastError();
                }
                if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
                if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
                float m = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&m, ev[0], ev[1]);
                tf += m;
                a = b;
                b = 1 - b;
                ++c->steps;
            }
            if (e == hipSuccess) {
                SweepArgs<S> sh{G(c, a), G(c, b), phi(c, b), nullptr, u(c), c->g, ph};
                launch_hydro(c, sh);
                e = hipGetLastError();
                c->cur = b;
                ++c->steps;
            }
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            for (int k = 0; k < 2; ++k) (void)hipEventDestroy(ev[k]);
            if (e != hipSuccess) return fail(LBM_EHIP, "timed fused steps failed: %s", hipGetErrorString(e));
            *fused_ms = tf / (n - 1);
            return LBM_OK;
        }
    }

    static lbm_status reduce(lbm_ctx *c, int mass_only, double out[kRedVals])
    {
        double *partial = (double *)(c->ws + c->L.off_red);
        double *dout = (double *)(c->ws + c->L.off_out);
        hipLaunchKernelGGL((k_reduce1<S>), dim3(kRedBlocks), dim3(kBlock), 0, c->stream, phi(c, c->cur), u(c),
                           c->g, make_phys<R>(&c->p), mass_only, partial);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(kBlock), 0, c->stream, partial, dout);
        LAUNCH_CHECK();
        HIP_TRY(hipMemcpyAsync(out, dout, kRedVals * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        return LBM_OK;
    }

    static lbm_status get_pdfs(lbm_ctx *c, double *Ho, double *Go)
    {
        hipLaunchKernelGGL((k_get_pdfs<S>), dim3(blocks(c)), dim3(kBlock), 0, c->stream, H(c, c->cur),
                           G(c, c->cur), phi(c, c->cur), Ho, Go, c->g, make_phys<R>(&c->p));
        LAUNCH_CHECK();
        return LBM_OK;
    }

    static lbm_status set_pdfs(lbm_ctx *c, const double *Hi, const double *Gi, const double *phi_i,
                               const double *u_i)
    {
        lbm_status s = zero_all(c);
        if (s != LBM_OK) return s;
        c->cur = 0;
        hipLaunchKernelGGL((k_set_pdfs<S>), dim3(blocks(c)), dim3(kBlock), 0, c->stream, H(c, 0), G(c, 1),
                           phi(c, 0), u(c), Hi, Gi, phi_i, u_i, c->g, make_phys<R>(&c->p));
        LAUNCH_CHECK();
        hipLaunchKernelGGL((k_unpull<S>), dim3(blocks(c)), dim3(kBlock), 0, c->stream, G(c, 1), G(c, 0), c->g);
        LAUNCH_CHECK();
        c->initialized = true;
        c->steps = 0;
        return LBM_OK;
    }

    template <class Out>
    static lbm_status get_macro(lbm_ctx *c, Out *phi_o, Out *u_o, Out *p_o)
    {
        hipLaunchKernelGGL((k_get_macro<S, Out>), dim3(blocks(c)), dim3(kBlock), 0, c->stream, G(c, c->cur),
                           phi(c, c->cur), u(c), phi_o, u_o, p_o, c->g, make_phys<R>(&c->p));
        LAUNCH_CHECK();
        return LBM_OK;
    }
};

template <template <class> class F, class B, class... A>
lbm_status dispatch_lattice(int variant, A &&...args)
{
    switch (variant) {
    case 0: return F<B>::run(args...);
    case 1: return F<Lattice<B, 15, 27, true>>::run(args...);
    case 2: return F<Lattice<B, 19, 19, false>>::run(args...);
    case 3: return F<Lattice<B, 19, 19, true>>::run(args...);
    case 4: return F<Lattice<B, 27, 27, false>>::run(args...);
    case 5: return F<Lattice<B, 15, 15, false>>::run(args...);
    }
    return fail(LBM_EARG, "lattice variant %d is not built", variant);
}

template <template <class> class F, class... A>
lbm_status dispatch(const lbm_params &p, A &&...args)
{
    const int variant = lattice_variant(&p);
    switch (p.storage) {
    case LBM_F64: return dispatch_lattice<F, StoreF64>(variant, args...);
    case LBM_F32: return dispatch_lattice<F, StoreF32>(variant, args...);
    case LBM_F16S: return F<StoreF16S>::run(args...);
    case LBM_BF16S: return F<StoreBF16S>::run(args...);
    }
    return fail(LBM_EARG, "unknown storage %d", p.storage);
}

template <class S> struct DoStep {
    static lbm_status run(lbm_ctx *c, int n) { return Ops<S>::step(c, n); }
};
template <class S> struct DoStepStraightforward {
    static lbm_status run(lbm_ctx *c, int n) { return Ops<S>::step_straightforward(c, n); }
};
template <class S> struct DoStepTimed {
    static lbm_status run(lbm_ctx *c, int n, double *a, double *b) { return Ops<S>::step_timed(c, n, a, b); }
};
template <class S> struct DoStepTimedFused {
    static lbm_status run(lbm_ctx *c, int n, double *f) { return Ops<S>::step_timed_fused(c, n, f); }
};
template <class S> struct DoReduce {
    static lbm_status run(lbm_ctx *c, int m, double *o) { return Ops<S>::reduce(c, m, o); }
};
template <class S> struct DoGetPdfs {
    static lbm_status run(lbm_ctx *c, double *H, double *G) { return Ops<S>::get_pdfs(c, H, G); }
};
template <class S> struct DoSetPdfs {
    static lbm_status run(lbm_ctx *c, const double *H, const double *G, const double *p, const double *u)
    {
        return Ops<S>::set_pdfs(c, H, G, p, u);
    }
};
template <class S> struct DoInit {
    static lbm_status run(lbm_ctx *c, const double *phi, const double *u, const double *ps)
    {
        return Ops<S>::template equilibrium<double>(c, phi, u, ps, 0);
    }
};
template <class S> struct DoSetMacro {
    static lbm_status run(lbm_ctx *c, int dtype, const void *phi, const void *u, const void *p)
    {
        if (dtype == LBM_DTYPE_F64)
            return Ops<S>::template equilibrium<double>(c, (const double *)phi, (const double *)u,
                                                        (const double *)p, 1);
        return Ops<S>::template equilibrium<float>(c, (const float *)phi, (const float *)u, (const float *)p, 1);
    }
};
template <class S> struct DoShiftEq {
    static lbm_status run(lbm_ctx *c, int dtype, const void *phi, const void *u, const void *p)
    {
        if (dtype == LBM_DTYPE_F64)
            return Ops<S>::template shift_equilibrium<double>(c, (const double *)phi, (const double *)u,
                                                              (const double *)p);
        return Ops<S>::template shift_equilibrium<float>(c, (const float *)phi, (const float *)u, (const float *)p);
    }
};
template <class S> struct DoGetMacro {
    static lbm_status run(lbm_ctx *c, int dtype, void *phi, void *u, void *p)
    {
        if (dtype == LBM_DTYPE_F64) return Ops<S>::get_macro(c, (double *)phi, (double *)u, (double *)p);
        return Ops<S>::get_macro(c, (float *)phi, (float *)u, (float *)p);
    }
};

lbm_status check_ctx(const lbm_ctx *c, bool need_init)
{
    if (!c) return fail(LBM_EARG, "context is NULL");
    if (need_init && !c->initialized) return fail(LBM_ESTATE, "state not initialised (call lbm_init_fields)");
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_velocity_set(int32_t q, int32_t *e, double *w)
{
    if (!e || !w) return fail(LBM_EARG, "NULL output");
    if (q != 15 && q != 19 && q != 27) return fail(LBM_EARG, "q must be 15, 19 or 27 (got %d)", q);
    for (int i = 0; i < q; ++i) {
        for (int a = 0; a < 3; ++a) e[3 * i + a] = q == 15 ? ev<15>(i, a) : ev<27>(i, a);
        w[i] = q == 15 ? wgt<15, double>(i) : q == 19 ? wgt<19, double>(i) : wgt<27, double>(i);
    }
    return LBM_OK;
}

size_t lbm_workspace_bytes(const lbm_params *p)
{
    if (validate(p) != LBM_OK) return 0;
    return layout(p).total;
}

lbm_status lbm_create(const lbm_params *p, void *ws, size_t bytes, void *stream, lbm_ctx **out)
{
    if (!out) return fail(LBM_EARG, "out is NULL");
    *out = nullptr;
    lbm_status s = validate(p);
    if (s != LBM_OK) return s;
    Layout L = layout(p);
    if (!ws) return fail(LBM_EARG, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(LBM_EARG, "workspace must be %zu-byte aligned", kAlign);
    if (bytes < L.total) return fail(LBM_ESIZE, "workspace has %zu bytes, needs %zu", bytes, L.total);
    lbm_ctx *c = new (std::nothrow) lbm_ctx;
    if (!c) return fail(LBM_EARG, "out of host memory");
    c->p = *p;
    c->stream = (hipStream_t)stream;
    c->ws = (char *)ws;
    c->ws_bytes = bytes;
    c->L = L;
    c->g.nx = p->nx;
    c->g.ny = p->ny;
    c->g.nz = p->nz;
    c->g.walls = p->walls_y ? 1 : 0;
    c->g.ncells = (int)L.ncells;
    c->g.half = (int)((L.ncells + 1) / 2);
    c->g.fplane = L.fplane;
    c->g.dnx = make_fastdiv((uint32_t)p->nx);
    c->g.dny = make_fastdiv((uint32_t)p->ny);
    c->cur = 0;
    c->initialized = false;
    c->steps = 0;
    c->zmarch = LBM_ZMARCH != 0;
    if (const char *v = std::getenv("LBM_ZMARCH")) c->zmarch = (v[0] == '1');
    c->pair16 = true;
    if (const char *v = std::getenv("LBM_PAIR")) c->pair16 = (v[0] != '0');
    c->fuse = true;
    if (const char *v = std::getenv("LBM_FUSE")) c->fuse = (v[0] != '0');
    *out = c;
    g_err[0] = 0;
    return LBM_OK;
}

lbm_status lbm_set_stream(lbm_ctx *c, void *stream)
{
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    c->stream = (hipStream_t)stream;
    return LBM_OK;
}

lbm_status lbm_init_fields(lbm_ctx *c, const double *phi, const double *u, const double *ps)
{
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (!phi || !u || !ps) return fail(LBM_EARG, "NULL field pointer");
    return dispatch<DoInit>(c->p, c, phi, u, ps);
}

lbm_status lbm_step(lbm_ctx *c, int32_t n)
{
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (n < 1) return fail(LBM_EARG, "n must be >= 1 (got %d)", n);
    return dispatch<DoStep>(c->p, c, (int)n);
}

lbm_status lbm_step_straightforward(lbm_ctx *c, int32_t n)
{
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (n < 1) return fail(LBM_EARG, "n must be >= 1 (got %d)", n);
    return dispatch<DoStepStraightforward>(c->p, c, (int)n);
}

lbm_status lbm_step_timed(lbm_ctx *c, int32_t n, double *phase_ms, double *hydro_ms)
{
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (n < 1 || n > 4096) return fail(LBM_EARG, "n must be in [1, 4096] (got %d)", n);
    if (!phase_ms || !hydro_ms) return fail(LBM_EARG, "NULL output");
    return dispatch<DoStepTimed>(c->p, c, (int)n, phase_ms, hydro_ms);
}

lbm_status lbm_step_timed_fused(lbm_ctx *c, int32_t n, double *fused_ms)
{
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (n < 2 || n > 4096) return fail(LBM_EARG, "n must be in [2, 4096] (got %d)", n);
    if (!fused_ms) return fail(LBM_EARG, "NULL output");
    return dispatch<DoStepTimedFused>(c->p, c, (int)n, fused_ms);
}

lbm_status lbm_reduce_mass(lbm_ctx *c, double *sum_phi)
{
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (!sum_phi) return fail(LBM_EARG, "NULL output");
    double v[kRedVals];
    s = dispatch<DoReduce>(c->p, c, 1, v);
    if (s != LBM_OK) return s;
    *sum_phi = v[0];
    if (!std::isfinite(v[0])) return fail(LBM_ENONFINITE, "sum of phi is not finite");
    return LBM_OK;
}

lbm_status lbm_reduce_stats(lbm_ctx *c, lbm_stats *o)
{
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (!o) return fail(LBM_EARG, "NULL output");
    double v[kRedVals];
    s = dispatch<DoReduce>(c->p, c, 0, v);
    if (s != LBM_OK) return s;
    std::memset(o, 0, sizeof(*o));
    o->mass = v[0];
    o->momentum[0] = v[1];
    o->momentum[1] = v[2];
    o->momentum[2] = v[3];
    o->gas_volume = v[4];
    if (v[4] != 0.0) {
        o->centroid[0] = v[5] / v[4];
        o->centroid[1] = v[6] / v[4];
        o->centroid[2] = v[7] / v[4];
        o->rise_velocity = v[8] / v[4];
    }
    o->interface_sum = v[9];
    o->grad_sum = v[10];
    o->xi_eff = v[10] != 0.0 ? v[9] / v[10] : 0.0;
    o->max_speed = v[11];
    for (int k = 0; k < kRedVals; ++k)
        if (!std::isfinite(v[k])) return fail(LBM_ENONFINITE, "reduction %d is not finite", k);
    return LBM_OK;
}

lbm_status lbm_get_macroscopic(lbm_ctx *c, int32_t dtype, void *phi, void *u, void *p)
{
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_F32) return fail(LBM_EARG, "unknown dtype %d", dtype);
    return dispatch<DoGetMacro>(c->p, c, (int)dtype, phi, u, p);
}

lbm_status lbm_set_macroscopic(lbm_ctx *c, int32_t dtype, const void *phi, const void *u, const void *p)
{
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_F32) return fail(LBM_EARG, "unknown dtype %d", dtype);
    if (!phi || !u || !p) return fail(LBM_EARG, "NULL field pointer");
    return dispatch<DoSetMacro>(c->p, c, (int)dtype, phi, u, p);
}

lbm_status lbm_shift_equilibrium(lbm_ctx *c, int32_t dtype, const void *phi, const void *u, const void *p)
{
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_F32) return fail(LBM_EARG, "unknown dtype %d", dtype);
    if (!phi || !u || !p) return fail(LBM_EARG, "NULL field pointer");
    return dispatch<DoShiftEq>(c->p, c, (int)dtype, phi, u, p);
}

lbm_status lbm_get_pdfs(lbm_ctx *c, double *H, double *G)
{
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    return dispatch<DoGetPdfs>(c->p, c, H, G);
}

lbm_status lbm_set_pdfs(lbm_ctx *c, const double *H, const double *G, const double *phi, const double *u)
{
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (!H || !G || !phi || !u) return fail(LBM_EARG, "NULL field pointer");
    return dispatch<DoSetPdfs>(c->p, c, H, G, phi, u);
}

lbm_status lbm_stream_copy(const void *src, void *dst, size_t bytes, void *stream)
{
    if (!src || !dst) return fail(LBM_EARG, "NULL buffer");
    if (bytes % 16) return fail(LBM_EARG, "bytes must be a multiple of 16");
    if (((uintptr_t)src) % 16 || ((uintptr_t)dst) % 16) return fail(LBM_EARG, "buffers must be 16-byte aligned");
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return LBM_OK;
    const int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 0x7fffffff) return fail(LBM_EARG, "copy of %zu bytes is too large", bytes);
    hipLaunchKernelGGL(k_copy, dim3((unsigned)nb), dim3(kBlock), 0, (hipStream_t)stream, (const uint4 *)src,
                       (uint4 *)dst, n);
    LAUNCH_CHECK();
    return LBM_OK;
}

static void state_parts(const lbm_ctx *c, size_t sz[4], size_t off_dst[5])
{
    const size_t pb = pdf_bytes(c->p.storage), rb = real_bytes(c->p.storage);
    sz[0] = (size_t)q_phase(&c->p) * (size_t)c->L.pdf_elems * pb;
    sz[1] = (size_t)q_hydro(&c->p) * (size_t)c->L.pdf_elems * pb;
    sz[2] = (size_t)c->L.fplane * rb;
    sz[3] = 3 * (size_t)c->L.fplane * rb;
    off_dst[0] = 0;
    for (int k = 0; k < 4; ++k) off_dst[k + 1] = align_up(off_dst[k] + sz[k], kAlign);
}

size_t lbm_state_bytes(const lbm_ctx *c)
{
    if (!c) return 0;
    size_t sz[4], off[5];
    state_parts(c, sz, off);
    return off[4];
}

lbm_status lbm_save_state(lbm_ctx *c, void *dst)
{
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (!dst || ((uintptr_t)dst) % kAlign) return fail(LBM_EARG, "dst must be a 256-byte aligned device pointer");
    size_t sz[4], off[5];
    state_parts(c, sz, off);
    const int k = c->cur;
    const char *src[4] = {c->ws + c->L.off_H[k], c->ws + c->L.off_G[k], c->ws + c->L.off_phi[k], c->ws + c->L.off_u};
    for (int i = 0; i < 4; ++i)
        HIP_TRY(hipMemcpyAsync((char *)dst + off[i], src[i], sz[i], hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
}

lbm_status lbm_restore_state(lbm_ctx *c, const void *src)
{
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (!src || ((uintptr_t)src) % kAlign) return fail(LBM_EARG, "src must be a 256-byte aligned device pointer");
    size_t sz[4], off[5];
    state_parts(c, sz, off);
    char *dst[4] = {c->ws + c->L.off_H[0], c->ws + c->L.off_G[0], c->ws + c->L.off_phi[0], c->ws + c->L.off_u};
    for (int i = 0; i < 4; ++i)
        HIP_TRY(hipMemcpyAsync(dst[i], (const char *)src + off[i], sz[i], hipMemcpyDeviceToDevice, c->stream));
    c->cur = 0;
    c->initialized = true;
    return LBM_OK;
}

int64_t lbm_steps_done(const lbm_ctx *c) { return c ? c->steps : -1; }

void lbm_destroy(lbm_ctx *c) { delete c; }

const char *lbm_last_error(void) { return g_err; }

}  // extern "C"
