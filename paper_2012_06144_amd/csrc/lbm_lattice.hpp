// Velocity sets, weights and storage codecs for the gfx950 sweeps.
//
// D3Q15 (phase field) and D3Q27 (hydrodynamics), Section 3 of Holzer et
// al. (IJHPCA 2020).  The weights are not printed in the paper; they are
// the standard isotropic sets (sum w = 1, sum w e e = I/3, fourth-order
// isotropy), spelled out here.  Canonical order: rest, axis pairs, edge
// pairs (D3Q27 only), corner pairs; the opposite of odd i is i+1.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

__host__ __device__ constexpr int e15(int i, int a)
{
    constexpr int T[15][3] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
        {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
    return T[i][a];
}

__host__ __device__ constexpr int e27(int i, int a)
{
    constexpr int T[27][3] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
        {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
        {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
        {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
    return T[i][a];
}

// D3Q19 is the rest, axis and edge part of D3Q27: its directions are the
// first 19 of the D3Q27 order.
template <int Q>
__host__ __device__ constexpr int ev(int i, int a)
{
    return Q == 15 ? e15(i, a) : e27(i, a);
}

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

template <int Q>
__host__ __device__ constexpr int l1(int i)
{
    return (ev<Q>(i, 0) != 0) + (ev<Q>(i, 1) != 0) + (ev<Q>(i, 2) != 0);
}

// Weight of direction i as a value of type R (divisions done in R).
template <int Q, class R>
__host__ __device__ constexpr R wgt(int i)
{
    return Q == 15   ? (l1<15>(i) == 0 ? R(2) / R(9) : l1<15>(i) == 1 ? R(1) / R(9) : R(1) / R(72))
           : Q == 19 ? (l1<19>(i) == 0 ? R(1) / R(3) : l1<19>(i) == 1 ? R(1) / R(18) : R(1) / R(36))
                     : (l1<27>(i) == 0 ? R(8) / R(27)
                        : l1<27>(i) == 1 ? R(2) / R(27)
                        : l1<27>(i) == 2 ? R(1) / R(54)
                                         : R(1) / R(216));
}

// ---- storage codecs ---------------------------------------------------------
// pdf_t: element type of the PDF planes; real: arithmetic type of the sweeps
// (also the type of the phi and u fields).  The 16-bit codecs (lowp) do not
// store the populations themselves but small numbers of order u:
//   phase field:  h_i - phi(cell) w_i   (decoded with the phi of the cell the
//                 population was stored at, which the stencil loads anyway)
//   hydrodynamic: g_i / w_i            (1/w_i is exact in binary)
// FP16 values are further scaled by 2^10 (exact) so that deviations down to
// ~1e-8 stay in the normal range of the format instead of its subnormals,
// whose coarse spacing would round the small same-signed bulk deviations
// with a bias.  BF16 has the exponent range of FP32 and needs no scaling.
// Rounding is to nearest even.
struct StoreF64 {
    static constexpr int QP = 15, QH = 27;  // velocity sets of the phase-field and hydrodynamic steps
    static constexpr bool phase_mrt = false;  // raw-moment MRT phase-field collision
    using pdf_t = double;
    using real = double;
    static constexpr bool lowp = false;
    static constexpr bool paired = false;  // cell c and c + half share a 32-bit word
    static constexpr real kScale = 1;
    __device__ static real ld(pdf_t v) { return v; }
    __device__ static pdf_t st(real v) { return v; }
};

struct StoreF32 {
    static constexpr int QP = 15, QH = 27;  // velocity sets of the phase-field and hydrodynamic steps
    static constexpr bool phase_mrt = false;  // raw-moment MRT phase-field collision
    using pdf_t = float;
    using real = float;
    static constexpr bool lowp = false;
    static constexpr bool paired = false;  // cell c and c + half share a 32-bit word
    static constexpr real kScale = 1;
    __device__ static real ld(pdf_t v) { return v; }
    __device__ static pdf_t st(real v) { return v; }
};

struct StoreF16S {
    static constexpr int QP = 15, QH = 27;  // velocity sets of the phase-field and hydrodynamic steps
    static constexpr bool phase_mrt = false;  // raw-moment MRT phase-field collision
    using pdf_t = __half;
    using real = float;
    static constexpr bool lowp = true;
    static constexpr bool paired = true;  // cell c and c + half share a 32-bit word
    static constexpr float kScale = 0x1p10f;  // stored = value * kScale
    __device__ static real raw_ld(pdf_t v) { return __half2float(v); }
    __device__ static pdf_t raw_st(real v) { return __float2half_rn(v); }
    __device__ static real ld(pdf_t v) { return raw_ld(v) * (1.0f / kScale); }
    __device__ static pdf_t st(real v) { return raw_st(v * kScale); }
};

struct StoreBF16S {
    static constexpr int QP = 15, QH = 27;  // velocity sets of the phase-field and hydrodynamic steps
    static constexpr bool phase_mrt = false;  // raw-moment MRT phase-field collision
    using pdf_t = __hip_bfloat16;
    using real = float;
    static constexpr bool lowp = true;
    static constexpr bool paired = true;  // cell c and c + half share a 32-bit word
    static constexpr float kScale = 1.0f;
    __device__ static real raw_ld(pdf_t v) { return __bfloat162float(v); }
    __device__ static pdf_t raw_st(real v) { return __float2bfloat16(v); }
    __device__ static real ld(pdf_t v) { return raw_ld(v); }
    __device__ static pdf_t st(real v) { return raw_st(v); }
};

// A storage type with other velocity sets (the stencil study of Sec. 5.1 and
// the D3Q19 lattice of Sec. 6.1) and optionally the raw-moment MRT of the
// phase field (Sec. 3.1).  FP64 and FP32 storage only.
template <class B, int QP_, int QH_, bool MRT_>
struct Lattice : B {
    static_assert(!B::lowp, "16-bit storage keeps D3Q15 / D3Q27");
    static_assert((QP_ == 15 || QP_ == 19 || QP_ == 27) && (QH_ == 15 || QH_ == 19 || QH_ == 27), "velocity set");
    static constexpr int QP = QP_, QH = QH_;
    static constexpr bool phase_mrt = MRT_;
};

// 1/w_i of D3Q27 (all exact in binary): 27/8, 27/2, 54, 216.
template <class R>
__host__ __device__ constexpr R inv_w27(int i)
{
    return l1<27>(i) == 0 ? R(3.375) : l1<27>(i) == 1 ? R(13.5) : l1<27>(i) == 2 ? R(54) : R(216);
}

// D3Q27 weight of the class of directions with k non-zero components.
template <class R>
__host__ __device__ constexpr R class_w27(int k)
{
    return k == 0 ? R(8) / R(27) : k == 1 ? R(2) / R(27) : k == 2 ? R(1) / R(54) : R(1) / R(216);
}

// Phase-field population i stored at a cell whose phase field is phi_cell.
template <class S>
__device__ inline typename S::pdf_t enc_h(typename S::real h, typename S::real phi_cell, int i)
{
    using R = typename S::real;
    if constexpr (S::lowp) return S::st(h - phi_cell * wgt<S::QP, R>(i));
    else return S::st(h);
}
template <class S>
__device__ inline typename S::real dec_h(typename S::pdf_t v, typename S::real phi_cell, int i)
{
    using R = typename S::real;
    if constexpr (S::lowp) return S::ld(v) + phi_cell * wgt<S::QP, R>(i);
    else return S::ld(v);
}
// Mass-budget forms of the phase-field codec for the FP32 and 16-bit paths:
// the decoded value in FP64 (the same operations wherever a population is
// decoded, so both sides of a sweep see identical numbers) and the encoding
// of an FP64 value with a single rounding to the storage type.
template <class S>
__device__ inline double dec_h64(typename S::pdf_t v, typename S::real phi_cell, int i)
{
    if constexpr (S::lowp) return double(S::ld(v)) + double(phi_cell) * wgt<S::QP, double>(i);
    else return double(S::ld(v));
}
template <class S>
__device__ inline typename S::pdf_t enc_h64(double h, typename S::real phi_cell, int i)
{
    using R = typename S::real;
    if constexpr (S::lowp) return S::st(R(h - double(phi_cell) * wgt<S::QP, double>(i)));
    else return S::st(R(h));
}
template <class S>
__device__ inline typename S::pdf_t enc_g(typename S::real g, int i)
{
    using R = typename S::real;
    if constexpr (S::lowp) return S::st(g * inv_w27<R>(i));
    else return S::st(g);
}
template <class S>
__device__ inline typename S::real dec_g(typename S::pdf_t v, int i)
{
    using R = typename S::real;
    if constexpr (S::lowp) return S::ld(v) * wgt<27, R>(i);  // stored g / w_i, decoded with the rounded w_i
    else return S::ld(v);
}

// ---- streaming memory access ---------------------------------------------------
// PDFs are touched once per sweep; LBM_NT_LOAD / LBM_NT_STORE mark those
// accesses non-temporal so they do not displace the phase-field rows the
// stencils re-read from L2.
#ifndef LBM_NT_LOAD
#define LBM_NT_LOAD 0
#endif
#ifndef LBM_NT_STORE
#define LBM_NT_STORE 1
#endif
#ifndef LBM_NT_FIELD
#define LBM_NT_FIELD 1
#endif

template <class T>
__device__ inline T ld_stream(const T *p)
{
    if constexpr (LBM_NT_LOAD && (sizeof(T) == 4 || sizeof(T) == 8) && !__is_class(T)) {
        return __builtin_nontemporal_load(p);
    } else if constexpr (LBM_NT_LOAD && sizeof(T) == 2) {
        const unsigned short v = __builtin_nontemporal_load(reinterpret_cast<const unsigned short *>(p));
        return __builtin_bit_cast(T, v);
    } else {
        return *p;
    }
}

template <class T>
__device__ inline void st_stream(T *p, T v)
{
    if constexpr (LBM_NT_STORE && (sizeof(T) == 4 || sizeof(T) == 8) && !__is_class(T)) {
        __builtin_nontemporal_store(v, p);
    } else if constexpr (LBM_NT_STORE && sizeof(T) == 2) {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v), reinterpret_cast<unsigned short *>(p));
    } else {
        *p = v;
    }
}

template <class T>
__device__ inline void st_field(T *p, T v)
{
    if constexpr (LBM_NT_FIELD) {
        __builtin_nontemporal_store(v, p);
    } else {
        *p = v;
    }
}

}  // namespace lbm
