// Device routines shared by the Couette and channel stage kernels: deterministic
// wavefront reductions, the WENO-5 face value, equilibrium expansion coefficients and
// the relaxation time.  Header-only (inline / internal linkage per translation unit).
#pragma once

#include <hip/hip_runtime.h>

#include "vlb_internal.h"

namespace vlb {

// Lane permutation of a double by a DPP control (applied to both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long x = __double_as_longlong(v);
    // every lane's source lane exists for the permutations used here (quad permutes and
    // mirrors within a row), so no fallback value is needed
    const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)x, l);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wavefront, returned in every lane, in a fixed order:
// quad butterflies (xor 1, xor 2) and the half-row and row mirrors by DPP give every
// lane its 16-lane row total; the four row totals are then added in lane order.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum over each 16-lane row of a wavefront (the row total in every lane of the row), in
// a fixed order: quad butterflies and the half-row and row mirrors by DPP.
__device__ __forceinline__ double row_sum(double v) {
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    v += dpp_mov<0x140>(v);
    return v;
}

// Row totals of four quantities at once (a transposed reduction): lane l holds the four
// products x_q = c_q v, q = 0..3, as k1 = x_{q(l)}, k2 = x_{q(l)^2}, s1 = x_{q(l)^1},
// s2 = x_{q(l)^3} with q(l) = l & 3.  A quad butterfly (xor 1) leaves each lane the pair
// sums of its own quantity and of the one its xor-2 partner keeps, a second (xor 2) the
// quad sum of its own quantity, and row rotations by 4 and 8 (which keep a lane's place in
// its quad) add the four quads: lane l returns the row total of quantity l & 3, in a fixed
// order.  Five adds and ten moves, against sixteen and thirty-two for four row_sum calls.
__device__ __forceinline__ double row_sum4(double k1, double k2, double s1, double s2) {
    const double a1 = k1 + dpp_mov<0xB1>(s1);   // quad_perm [1,0,3,2]
    const double a2 = k2 + dpp_mov<0xB1>(s2);
    double b = a1 + dpp_mov<0x4E>(a2);          // quad_perm [2,3,0,1]
    b += dpp_mov<0x124>(b);                     // row_ror:4
    b += dpp_mov<0x128>(b);                     // row_ror:8
    return b;
}

// Raw buffer access (range-checked by the resource): an offset at or beyond the resource's
// byte count reads 0 and drops the write, so loads and stores of lanes with nothing to
// move are still issued, and every wavefront issues the same memory instructions in the
// same order (the compiler then waits for a load by its position in that order, not for
// every outstanding access).
constexpr unsigned kBufNone = 0x80000000u;   // an offset outside every resource
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// voff: the lane's byte offset (kBufNone for a lane with nothing to move); soff: a
// wavefront-uniform byte offset added to it (kept in a scalar register).
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff = 0);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, 0);
}

// 1/x: the hardware reciprocal in FP32 (about 1 ulp, the FP32 path's tolerance is far
// wider); in FP64 the hardware estimate refined by two Newton steps r <- r + r (1 - x r)
// (each squares the relative error; the result is within an ulp or so of 1/x, for the
// normal, positive arguments the WENO weights take; x = 0 gives NaN, like 0 * (1/0)).
template <typename T>
__device__ __forceinline__ T recip(T x);
template <>
__device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double recip<double>(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Flux at the face between c and d, upwinded from c (a, b, c, d, e in upwind order).
// GUARD (FP32): stencils whose values span more than the FP32 exponent range (the
// defect correction's corrections do, populations never) can underflow the weights;
// there the weights' limit is taken instead (see below).
template <typename T, bool GUARD = false>
__device__ __forceinline__ T weno5(T a, T b, T c, T d, T e, T eps);

// Face flux between window cells 2 and 3 of a six-cell window (cells s-2 .. s+3):
// upwinded from cell 2 when the advection velocity is positive, from cell 3 otherwise
// (the mirror image of the printed stencil).  The five stencil values are selected
// first, so a wavefront holding both signs evaluates WENO once.
template <typename T, bool GUARD = false>
__device__ __forceinline__ T weno_face(bool pos, T w0, T w1, T w2, T w3, T w4, T w5, T eps) {
    return weno5<T, GUARD>(pos ? w0 : w5, pos ? w1 : w4, pos ? w2 : w3, pos ? w3 : w2, pos ? w4 : w1, eps);
}

template <typename T, bool GUARD>
__device__ __forceinline__ T weno5(T a, T b, T c, T d, T e, T eps) {
    const T f1 = a * T(1.0 / 3.0) - b * T(7.0 / 6.0) + c * T(11.0 / 6.0);
    const T f2 = -b * T(1.0 / 6.0) + c * T(5.0 / 6.0) + d * T(1.0 / 3.0);
    const T f3 = c * T(1.0 / 3.0) + d * T(5.0 / 6.0) - e * T(1.0 / 6.0);
    T t1 = a - T(2) * b + c, t2 = a - T(4) * b + T(3) * c;
    T s1 = T(13.0 / 12.0) * (t1 * t1) + T(0.25) * (t2 * t2);
    t1 = b - T(2) * c + d;
    t2 = b - d;
    T s2 = T(13.0 / 12.0) * (t1 * t1) + T(0.25) * (t2 * t2);
    t1 = c - T(2) * d + e;
    t2 = T(3) * c - T(4) * d + e;
    T s3 = T(13.0 / 12.0) * (t1 * t1) + T(0.25) * (t2 * t2);
    // an indicator vanishes exactly when its three values are equal (Eq. weno_sigma is a
    // sum of squares of two independent differences); the equality test is immune to the
    // compiler fusing the products that form the values into the indicator arithmetic
    // (identical ghost values must select the Table weno limit, whatever eps)
    const bool z1 = (a == b && b == c) || s1 == T(0), z2 = (b == c && c == d) || s2 == T(0),
               z3 = (c == d && d == e) || s3 == T(0), zany = z1 || z2 || z3;
    if (eps != T(0)) {   // optional regularisation (eps is uniform over the instance)
        const T add = zany ? T(0) : eps * T(0.2) * (a * a + b * b + c * c + d * d + e * e);
        s1 += add;
        s2 += add;
        s3 += add;
    }
    // w_q proportional to d_q / s_q^2, rewritten as d_q (r_a r_b)^2 with r = s / max(s):
    // one division instead of three and no overflow.  In FP64 an underflow would need two
    // indicators below 1e-155 of the largest, which only exact zeros reach; the FP32 path
    // runs on populations scaled by 1/(w_i w_j), which are O(1), so its indicators stay
    // far from the FP32 range limits.  Exactly vanishing indicators take the limits of
    // Table weno instead (selected without branching; the unused product form may be NaN
    // when every indicator vanishes and is discarded by the select).
    T m = s1 > s2 ? s1 : s2;
    m = m > s3 ? m : s3;
    const T inv = recip<T>(m);
    const T r1 = s1 * inv, r2 = s2 * inv, r3 = s3 * inv;
    const T q23 = r2 * r3, q13 = r1 * r3, q12 = r1 * r2;
    const T w1 = zany ? (z1 ? T(0.1) : T(0)) : T(0.1) * (q23 * q23);
    const T w2 = zany ? (z2 ? T(0.6) : T(0)) : T(0.6) * (q13 * q13);
    const T w3 = zany ? (z3 ? T(0.3) : T(0)) : T(0.3) * (q12 * q12);
    const T sw = w1 + w2 + w3;
    if constexpr (GUARD) {
        // with two indicators below about 1e-19 of the largest (or the largest itself below
        // the normal range), the product form underflows; the normalised weights then tend
        // to 1 on the stencil of the smallest indicator, which is taken
        if (!zany && !(m >= T(1.17549435e-38f) && sw >= T(1.17549435e-38f)))
            return (s1 <= s2 && s1 <= s3) ? f1 : (s2 <= s3 ? f2 : f3);
    }
    return (w1 * f1 + w2 * f2 + w3 * f3) * recip<T>(sw);
}

// Expansion coefficients of one axis' equilibrium factor at (u, T) (Sec. IV.D):
// full range: coefficient of phi_l = He_l/sqrt(l!) is E[He_l(X)]/sqrt(l!), X ~ N(u, T),
//   with a_l = E[He_l]/l! from l a_l = u a_{l-1} + (T-1) a_{l-2};
// half range: coefficient of phi_l is sum_s C[l][s] M_s with the half-line moments
//   M_s = int_0^inf x^s N(x; +-u, T) dx:  M_0 = (1+erf(zeta))/2, M_1 = u M_0 + T g(0),
//   M_s = u M_{s-1} + (s-1) T M_{s-2}.  Writes plus- and minus-side coefficients.
// Loops run to the compile-time bound kMaxN with the order N as a guard, so the moments
// and the table entries live in registers (no per-lane scratch array) and the table loads
// are independent of one another; the sums keep their order.
__device__ __forceinline__ void half_line_moments(double uu, double T, double (&M)[kMaxN + 1]) {
    const double g0 = exp(-uu * uu / (2.0 * T)) / sqrt(2.0 * M_PI * T);
    M[0] = 0.5 * (1.0 + erf(uu / sqrt(2.0 * T)));
    M[1] = uu * M[0] + T * g0;
#pragma unroll
    for (int s = 2; s <= kMaxN; ++s) M[s] = uu * M[s - 1] + (s - 1) * T * M[s - 2];   // entries past N unused
}
// lower triangle of C (rows l <= N), row l at l (l + 1) / 2
__device__ __forceinline__ void load_half_table(const double* C, int N, double (&Ct)[(kMaxN + 1) * (kMaxN + 2) / 2]) {
#pragma unroll
    for (int l = 0; l <= kMaxN; ++l)
#pragma unroll
        for (int s = 0; s <= l; ++s) Ct[l * (l + 1) / 2 + s] = l <= N ? C[l * (N + 1) + s] : 0.0;
}
__device__ __forceinline__ void half_coef(int N, const double (&Ct)[(kMaxN + 1) * (kMaxN + 2) / 2],
                                          const double (&M)[kMaxN + 1], double* co) {
#pragma unroll
    for (int l = 0; l <= kMaxN; ++l) {
        if (l > N) break;
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s <= l; ++s) acc += Ct[l * (l + 1) / 2 + s] * M[s];
        co[l] = acc;
    }
}
__device__ __forceinline__ void full_coef(int N, double u, double T, const double* isf, double* co) {
    double a0 = 1.0, a1 = u;
    co[0] = a0 / isf[0];
    if (N >= 1) co[1] = a1 / isf[1];
    for (int l = 2; l <= N; ++l) {
        const double a2 = (u * a1 + (T - 1.0) * a0) / l;
        co[l] = a2 / isf[l];
        a0 = a1;
        a1 = a2;
    }
}

static __device__ __noinline__ void axis_coef(int kind, int N, double u, double T, const double* C, const double* isf,
                          double* cp, double* cm) {
    if (kind == 0) {
        full_coef(N, u, T, isf, cp);
        for (int l = 0; l <= N; ++l) cm[l] = cp[l];
        return;
    }
    double Ct[(kMaxN + 1) * (kMaxN + 2) / 2];
    load_half_table(C, N, Ct);
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
        double M[kMaxN + 1];
        half_line_moments(sg == 0 ? u : -u, T, M);
        half_coef(N, Ct, M, sg == 0 ? cp : cm);
    }
}

// One side of axis_coef: for a half-range axis (kind 1) the coefficients of the side sg
// (0: +u, 1: -u); for a full-range axis (kind 0) its coefficients (sg ignored).  Lanes of
// a wavefront that take different sides run the same instructions together.
static __device__ __noinline__ void axis_coef_side(int kind, int N, double u, double T, const double* C,
                                                   const double* isf, int sg, double* co) {
    if (kind == 0) {
        full_coef(N, u, T, isf, co);
        return;
    }
    double Ct[(kMaxN + 1) * (kMaxN + 2) / 2];
    load_half_table(C, N, Ct);
    double M[kMaxN + 1];
    half_line_moments(sg == 0 ? u : -u, T, M);
    half_coef(N, Ct, M, co);
}

__device__ __forceinline__ double tau_of(int model, double Kn, double n, double T) {
    if (model == 0) return Kn * 0.62665706865775012 / n;   // Kn sqrt(pi/8)/n, Eq. tau_aoki
    if (model == 1) return Kn / (n * T);                   // Eq. hydro_tau
    return Kn / n;
}

}  // namespace vlb
