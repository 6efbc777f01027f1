// cse_flip.hpp -- random ternary flips of a matrix multiplication scheme
// (Sec. 3.5.3: M variants of the scheme, variant 0 the scheme itself, the
// others made by a random number of flips and regenerated every iteration).
//
// A scheme of format (n, m, p : r) is r products t = U_t (x) V_t (x) W_t of
// ternary vectors over the entries of A (n x m), B (m x p) and C (n x p).
// When two products i != j share a factor up to sign, X_j = s X_i (X one of
// U, V, W; s = +1 or -1), the identity
//   X_i(x)Y_i(x)Z_i + X_j(x)Y_j(x)Z_j = X_i(x)(Y_i + s Y_j)(x)Z_i + X_j(x)Y_j(x)(Z_j - Z_i)   (h = 0)
//                                     = X_i(x)Y_i(x)(Z_i + s Z_j) + X_j(x)(Y_j - Y_i)(x)Z_j   (h = 1)
// ((Y, Z) = (V, W), (U, W), (U, V) for X = U, V, W) rewrites the scheme into
// another one of the same rank computing the same product.  A flip is valid
// when both changed vectors stay ternary and nonzero; valid flips are
// numbered in the order (X, i, j, h).  Variant v != 0 at iteration `it`
// applies F = 1 + floor(u F_max / 2^32) flips, u word 0 of Philox block
// (v, FLIP|0|it|0, 0, 0); flip f takes valid flip floor(u' n_valid / 2^32)
// of the current scheme, u' word 0 of (v, FLIP|0|it|f+1, 0, 0), and the
// sequence stops early when no flip is valid.
//
// flip_variants_kernel: one workgroup (one wave) per variant; the variant's
// U, V and W live in LDS while its flips are drawn and applied.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cse_kernels.hpp"

namespace csek {

constexpr uint32_t TAG_FLIP = 6;

struct FlipArgs {
    const int8_t* U;  // r x nm
    const int8_t* V;  // r x mp
    const int8_t* W;  // r x np (the products' C coefficients)
    int8_t* outU;     // n_variants x r x nm
    int8_t* outV;
    int8_t* outW;
    int8_t* outWt;    // n_variants x np x r (the E_W system of each variant), or null
    int32_t* n_done;  // flips applied per variant
    int32_t r, len[3];
    uint32_t max_flips, iteration;
    uint64_t seed;
};

__host__ __device__ inline size_t flip_lds_bytes(int r, int lu, int lv, int lw) {
    return (((size_t)r * (lu + lv + lw)) + 15) & ~size_t(15);
}

// s with X_j = s X_i (X_i nonzero), else 0.
__device__ __forceinline__ int flip_sign(const int8_t* xi, const int8_t* xj, int len) {
    bool sp = true, sm = true, nz = false;
    for (int k = 0; k < len; ++k) {
        sp &= xj[k] == xi[k];
        sm &= xj[k] == -xi[k];
        nz |= xi[k] != 0;
    }
    return !nz ? 0 : sp ? 1 : sm ? -1 : 0;
}

// a + s b stays ternary and nonzero.
__device__ __forceinline__ bool flip_sum_ok(const int8_t* a, const int8_t* b, int s, int len) {
    bool ok = true, nz = false;
    for (int k = 0; k < len; ++k) {
        const int v = a[k] + s * b[k];
        ok &= v >= -1 && v <= 1;
        nz |= v != 0;
    }
    return ok && nz;
}

// Validity of flip (X, i, j, h = 0 and 1) with t = (X r + i) r + j: bit h.
__device__ __forceinline__ int flip_bits(int8_t* const M[3], const int len[3], int r, int t, int* sign) {
    const int X = t / (r * r), i = (t / r) % r, j = t % r;
    *sign = 0;
    if (i == j) return 0;
    const int Y = X == 0 ? 1 : 0, Z = X == 2 ? 1 : 2;
    const int s = flip_sign(M[X] + (size_t)i * len[X], M[X] + (size_t)j * len[X], len[X]);
    if (!s) return 0;
    *sign = s;
    const int8_t *Yi = M[Y] + (size_t)i * len[Y], *Yj = M[Y] + (size_t)j * len[Y];
    const int8_t *Zi = M[Z] + (size_t)i * len[Z], *Zj = M[Z] + (size_t)j * len[Z];
    const bool h0 = flip_sum_ok(Yi, Yj, s, len[Y]) && flip_sum_ok(Zj, Zi, -1, len[Z]);
    const bool h1 = flip_sum_ok(Zi, Zj, s, len[Z]) && flip_sum_ok(Yj, Yi, -1, len[Y]);
    return (h0 ? 1 : 0) | (h1 ? 2 : 0);
}

__global__ __launch_bounds__(kWave) void flip_variants_kernel(FlipArgs A) {
    extern __shared__ uint64_t smem[];
    const int l = lane_id();
    const int v = blockIdx.x, r = A.r;
    const int len[3] = {A.len[0], A.len[1], A.len[2]};
    int8_t* const M[3] = {(int8_t*)smem, (int8_t*)smem + (size_t)r * len[0],
                          (int8_t*)smem + (size_t)r * (len[0] + len[1])};
    const int8_t* const src[3] = {A.U, A.V, A.W};
    for (int x = 0; x < 3; ++x)
        for (int k = l; k < r * len[x]; k += kWave) M[x][k] = src[x][k];
    __syncthreads();
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    int done = 0;
    if (v != 0) {
        const U4 d = philox10((uint32_t)v, domain(TAG_FLIP, 0, A.iteration, 0), 0u, 0u, k0, k1);
        const uint32_t F = 1u + scale_u32(d.x, A.max_flips);
        const int n_t = 3 * r * r;
        for (uint32_t f = 0; f < F; ++f) {
            // Count the valid flips in order.
            int n_valid = 0;
            for (int base = 0; base < n_t; base += kWave) {
                int s;
                const int b = base + l < n_t ? flip_bits(M, len, r, base + l, &s) : 0;
                n_valid += wave_sum(__popc((unsigned)b));
            }
            if (n_valid == 0) break;
            const U4 e = philox10((uint32_t)v, domain(TAG_FLIP, 0, A.iteration, f + 1), 0u, 0u, k0, k1);
            const int want = (int)scale_u32(e.x, (uint32_t)n_valid);
            // Find it: the lane whose running count crosses `want`.
            int before = 0, t_sel = -1, h_sel = 0, s_sel = 0;
            for (int base = 0; base < n_t && t_sel < 0; base += kWave) {
                int s;
                const int t = base + l;
                const int b = t < n_t ? flip_bits(M, len, r, t, &s) : 0;
                const int c = __popc((unsigned)b);
                const int incl = wave_scan(c);
                const bool here = c > 0 && before + incl - c <= want && want < before + incl;
                const uint64_t hit = ballot(here);
                if (hit) {
                    const int src_l = ctz64(hit);
                    const int tt = __shfl(t, src_l), bb = __shfl(b, src_l), ss = __shfl(s, src_l);
                    const int ex = __shfl(before + incl - c, src_l);
                    // Bit h = 0 is numbered before h = 1.
                    const int hh = (want == ex && (bb & 1)) ? 0 : 1;
                    t_sel = tt;
                    h_sel = hh;
                    s_sel = ss;
                }
                before += __shfl(incl, kWave - 1);
            }
            const int X = t_sel / (r * r), i = (t_sel / r) % r, j = t_sel % r;
            const int Y = X == 0 ? 1 : 0, Z = X == 2 ? 1 : 2;
            // h = 0: Y_i += s Y_j, Z_j -= Z_i;  h = 1: Z_i += s Z_j, Y_j -= Y_i.
            const int P = h_sel ? Z : Y, Q = h_sel ? Y : Z;
            __syncthreads();
            for (int k = l; k < len[P]; k += kWave)
                M[P][(size_t)i * len[P] + k] = (int8_t)(M[P][(size_t)i * len[P] + k] + s_sel * M[P][(size_t)j * len[P] + k]);
            for (int k = l; k < len[Q]; k += kWave)
                M[Q][(size_t)j * len[Q] + k] = (int8_t)(M[Q][(size_t)j * len[Q] + k] - M[Q][(size_t)i * len[Q] + k]);
            __syncthreads();
            ++done;
        }
    }
    int8_t* const dst[3] = {A.outU + (size_t)v * r * len[0], A.outV + (size_t)v * r * len[1],
                            A.outW + (size_t)v * r * len[2]};
    for (int x = 0; x < 3; ++x)
        for (int k = l; k < r * len[x]; k += kWave) dst[x][k] = M[x][k];
    if (A.outWt) {
        int8_t* wt = A.outWt + (size_t)v * r * len[2];
        for (int k = l; k < r * len[2]; k += kWave) {
            const int c = k / r, t = k % r;  // W^T row c (an entry of C), column t (a product)
            wt[k] = M[2][(size_t)t * len[2] + c];
        }
    }
    if (l == 0) A.n_done[v] = done;
}

}  // namespace csek
