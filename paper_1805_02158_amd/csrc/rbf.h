// Influence function of the TNRD-style denoiser stage (Sec. IV names TNRD):
//   phi(z) = sum_j w_j exp(-(z - mu_j)^2 / (2 gamma^2)),  mu_j = mu0 + j dmu,
// evaluated exactly on the 2K+1 centres nearest z. With j0 the nearest centre, d0 = z - mu_j0,
// c = log2(e) / (2 gamma^2), A = exp2(2 c dmu d0), B = exp2(-c dmu^2), the term of centre
// j0 + k is w_{j0+k} G0 A^k B^(k^2), G0 = exp2(-c d0^2). Centres farther than K + 1/2
// spacings add less than eps of a weight: eps = 1e-12 in the FP32 form (K = 7 for gamma = dmu),
// 1e-6 in the BF16 form (K = 5), whose operands carry 3.9e-3 relative error.
//
// Compile-time window (K fixed): phi = G0 A^-K sum_{m=0}^{2K} c_|m-K| w_{j0+m-K} A^m by Horner
// in A, c_k = B^(k^2) precomputed, the prefactor one exp2 (two exp2 and 2K FMA + 2K+1
// multiplies per evaluation), with no branch: j0 is clamped to -K .. J-1+K, where the window's
// weights lie in the row's zero padding, and d0 to [-dmu, dmu]. Inside that range the sum is
// the window's exactly (j0 is the nearest centre up to rounding at a midpoint, where the window
// then misses a term beyond (K + 1/2) dmu); the d0 clamp binds only for z more than K + 1
// spacings beyond the first or last centre, where every term is below eps of a weight. With
// |d0| <= dmu every intermediate stays below 2^(4 K c dmu^2), far inside FP32 for the
// gamma / dmu the compile-time windows serve. Runtime K: the two-sided recurrence
// term(k+1) = term(k) R_k, R_{k+1} = R_k B^2, which stays bounded for any z; past the cut-off
// (K + 1/2) dmu every term is negligible and the result is 0.
//
// Tabulated form (BF16 stage): phi is read from a per-filter table of the cubic Hermite
// interpolant of the exact sum (all J terms, built in FP64 from phi and phi' at knots spaced
// gamma / 2), one interval of four coefficients per lookup: three FMAs instead of two exp2 and
// a 2K+1 term polynomial. Its error is at most h^4 / 384 max |phi''''| (h = gamma / 2: below
// 5e-4 of the local weight sum), an order below the 3.9e-3 of the BF16 operands.
#pragma once

#include <math.h>

#include "internal.h"

namespace redve {

struct RbfParams {
    float mu0, dmu, inv_dmu, half_dmu;
    float t0;      // -mu0 / dmu: (z - mu0) / dmu = z inv_dmu + t0
    float jlast;   // J - 1
    float c;       // log2(e) / (2 gamma^2)
    float two_cd;  // 2 c dmu
    float kpre;    // K 2 c dmu: the A^-K factor of the prefactor
    float b, b2;   // B and B^2 (recurrence)
    float cutoff;  // (K + 1/2) dmu
    float ck[kMaxRbfWindow + 1];  // B^(k^2), k = 0..K
    int J, K;
    // tabulated form: t = z t_scale + t_off = (z - lo) / h, intervals 0 .. t_last
    float t_scale, t_off, t_last;
    int tab_n;
};

inline RbfParams rbf_params(const TnrdDev& d) {
    RbfParams p{};
    p.mu0 = d.mu0;
    p.dmu = d.dmu;
    p.inv_dmu = 1.0f / d.dmu;
    p.half_dmu = 0.5f * d.dmu;
    p.t0 = (float)(-(double)d.mu0 / (double)d.dmu);
    p.jlast = (float)(d.nrbf - 1);
    const double c = 1.4426950408889634 / (2.0 * (double)d.gamma * d.gamma);
    const double cd2 = c * (double)d.dmu * d.dmu;
    p.c = (float)c;
    p.two_cd = (float)(2.0 * c * d.dmu);
    p.kpre = (float)(d.kwin * 2.0 * c * d.dmu);
    p.b = (float)exp2(-cd2);
    p.b2 = (float)exp2(-2.0 * cd2);
    p.cutoff = (float)(d.kwin + 0.5) * d.dmu;
    for (int k = 0; k <= kMaxRbfWindow; ++k) p.ck[k] = (float)exp2(-cd2 * k * k);
    p.J = d.nrbf;
    p.K = d.kwin;
    p.t_scale = d.tab_scale;
    p.t_off = d.tab_off;
    p.t_last = (float)(d.tab_n > 0 ? d.tab_n - 1 : 0);
    p.tab_n = d.tab_n;
    return p;
}

// Tabulated phi: tab holds the function's intervals as (a0, a1, a2, a3), 16-byte aligned.
// z below the table's range takes interval 0, above it the last (both below 1e-6 of a weight
// there); the index is clamped in floating point, so any z, NaN included, stays in the table.
__device__ inline float phi_table(float z, const float* tab, const RbfParams& p) {
    const float t = fmaf(z, p.t_scale, p.t_off);
    const float tf = floorf(t);
    const int k = (int)fminf(fmaxf(tf, 0.f), p.t_last);
    const float u = t - tf;
    const float4 c = *reinterpret_cast<const float4*>(tab + 4 * k);
    return fmaf(fmaf(fmaf(c.w, u, c.z), u, c.y), u, c.x);
}

// wrow: the function's weights with kRbfPad zeros on each side (the layout of
// TnrdDev::rbf_w). KC > 0: compile-time window (= p.K); KC = 0: any K <= kMaxRbfWindow,
// recurrence only.
template <int KC>
__device__ inline float phi_eval(float z, const float* wrow, const RbfParams& p) {
    if constexpr (KC > 0) {
        static_assert(2 * KC <= kRbfPad, "the clamped window stays inside the padded row");
        // nearest centre, clamped in floating point before the conversion, so that any z (NaN
        // and infinities included) reads inside the padded weight row
        const float jf =
            fminf(fmaxf(rintf(fmaf(z, p.inv_dmu, p.t0)), (float)-KC), p.jlast + (float)KC);
        const int j0 = (int)jf;
        const float d0 = fminf(fmaxf(z - fmaf(p.dmu, jf, p.mu0), -p.dmu), p.dmu);
        const float* wc = wrow + kRbfPad + j0;
        // the 2K+1 weights first, so their reads are in flight together ahead of the chain
        float wv[2 * KC + 1];
#pragma unroll
        for (int m = 0; m <= 2 * KC; ++m) wv[m] = wc[m - KC];
        const float a = __builtin_amdgcn_exp2f(p.two_cd * d0);
        const float pre = __builtin_amdgcn_exp2f(-(p.c * d0 + p.kpre) * d0);
        float poly = p.ck[KC] * wv[2 * KC];
#pragma unroll
        for (int m = 2 * KC - 1; m >= 0; --m) {
            const int k = m - KC;
            poly = fmaf(poly, a, p.ck[k < 0 ? -k : k] * wv[m]);
        }
        return pre * poly;
    } else {
        const int j0 = (int)fminf(fmaxf(rintf((z - p.mu0) * p.inv_dmu), 0.f), p.jlast);
        const float d0r = z - (p.mu0 + p.dmu * (float)j0);
        const float* wc = wrow + kRbfPad + j0;
        const int K = p.K;
        const bool live = fabsf(d0r) <= p.cutoff;
        const float d0 = live ? d0r : 0.f;
        const float g0 = live ? __builtin_amdgcn_exp2f(-p.c * d0 * d0) : 0.f;
        const float a = __builtin_amdgcn_exp2f(p.two_cd * d0);
        const float ai = __builtin_amdgcn_exp2f(-p.two_cd * d0);
        float acc = wc[0] * g0;
        float gu = g0, ru = a * p.b, gd = g0, rd = ai * p.b;
#pragma unroll
        for (int k = 1; k <= kMaxRbfWindow; ++k) {
            if (k > K) break;
            gu *= ru;
            ru *= p.b2;
            gd *= rd;
            rd *= p.b2;
            acc += wc[k] * gu + wc[-k] * gd;
        }
        return acc;
    }
}

}  // namespace redve
