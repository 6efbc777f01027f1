// cse_input.hpp -- Analysis of an input system on the device (Sec. 3.3,
// Algorithm 1's first Analysis), once per component: every process of a
// component starts from the same system, so its pair counts, candidate
// list and second ordering are computed once and copied by each unit.
//
//   input_columns_kernel   int8 rows x cols -> positive / negative column bitsets
//   input_features_kernel  the same as an int8 0/1 matrix [P N] (Gram path)
//   input_gram_kernel      G = [P N]^T [P N] on the int8 matrix cores
//   input_count_kernel     candidates per first variable / per second variable
//   input_scan_kernel      exclusive offsets of both, and the candidate count
//   input_rows_kernel      candidates in canonical order (key order)
//   input_cols_kernel      the second ordering: canonical indices by (second, first, sign)
//
// Pair counts (Sec. 3.3): c+(a, b) = |P_a & P_b| + |N_a & N_b|,
// c-(a, b) = |P_a & N_b| + |N_a & P_b|; the popcount path evaluates them on
// the bitsets, the Gram path reads them from G.  Both give the same integers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace csek {

constexpr int kInputBlock = 256;

// Counts of pair (a, b), a != b (0-based variables).
struct PairSource {
    const uint64_t* P;
    const uint64_t* N;
    int W;
    const int32_t* G;  // Gram path: (2 n_x padded) x same, row-major; null for popcount
    int F;             // row length of G
    int n_x;

    __device__ __forceinline__ int2 counts(int a, int b) const {
        if (G) {
            const size_t Fs = (size_t)F;
            const int cp = G[a * Fs + b] + G[(n_x + a) * Fs + (n_x + b)];
            const int cm = G[a * Fs + (n_x + b)] + G[(n_x + a) * Fs + b];
            return make_int2(cp, cm);
        }
        int cp = 0, cm = 0;
        for (int w = 0; w < W; ++w) {
            const uint64_t pa = P[(size_t)a * W + w], na = N[(size_t)a * W + w];
            const uint64_t pb = P[(size_t)b * W + w], nb = N[(size_t)b * W + w];
            cp += __popcll(pa & pb) + __popcll(na & nb);
            cm += __popcll(pa & nb) + __popcll(na & pb);
        }
        return make_int2(cp, cm);
    }
};

// Exclusive scan over a block of kInputBlock threads (4 waves); *total gets the sum.
__device__ __forceinline__ int block_exclusive_scan(int v, int* total) {
    __shared__ int wsum[kInputBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int before = 0, all = 0;
    for (int w = 0; w < kInputBlock / 64; ++w) {
        before += w < wave ? wsum[w] : 0;
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// Validation and sizes of a device-resident input (Sec. 3.2.1): per row its
// nonzeros r; st[0] += sum r, st[1] += sum r (r - 1) / 2 (pair occurrences),
// st[2] += sum (r - 1) (the naive count), st[3] counts entries outside
// {-1, 0, 1}, st[4] counts all-zero rows.  st starts at zero.
__global__ void input_stats_kernel(const int8_t* __restrict__ A, int rows, int cols, unsigned long long* st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    long long r = 0, bad = 0;
    for (int j = 0; j < cols; ++j) {
        const int v = A[(size_t)i * cols + j];
        r += v != 0;
        bad += v < -1 || v > 1;
    }
    atomicAdd(&st[0], (unsigned long long)r);
    atomicAdd(&st[1], (unsigned long long)(r * (r - 1) / 2));
    if (r > 0) atomicAdd(&st[2], (unsigned long long)(r - 1));
    if (bad) atomicAdd(&st[3], (unsigned long long)bad);
    if (r == 0) atomicAdd(&st[4], 1ull);
}

// P[v W + w] bit i: A[64 w + i][v] > 0; N likewise for < 0.
__global__ void input_columns_kernel(const int8_t* __restrict__ A, int rows, int cols, int W, uint64_t* P,
                                     uint64_t* N) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cols * W) return;
    const int v = t / W, w = t % W;
    uint64_t p = 0, n = 0;
    for (int i = 0; i < 64; ++i) {
        const int r = 64 * w + i;
        if (r < rows) {
            const int8_t x = A[(size_t)r * cols + v];
            p |= (uint64_t)(x > 0) << i;
            n |= (uint64_t)(x < 0) << i;
        }
    }
    P[t] = p;
    N[t] = n;
}

// X[f Kp + r] = 1 where feature f (P columns 0 .. n_x-1, then N columns)
// holds row r; rows padded to Kp, features to F, with zeros.
__global__ void input_features_kernel(const int8_t* __restrict__ A, int rows, int cols, int Kp, int F,
                                      int8_t* X) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)F * Kp) return;
    const int f = (int)(t / Kp), r = (int)(t % Kp);
    int8_t x = 0;
    if (r < rows && f < 2 * cols) {
        const int8_t a = A[(size_t)r * cols + (f < cols ? f : f - cols)];
        x = f < cols ? (int8_t)(a > 0) : (int8_t)(a < 0);
    }
    X[t] = x;
}

// G = X X^T over 32 x 32 tiles, one wave per tile: each step multiplies a
// 32 x 16 slab of the tile's rows by the same slab of its columns.  A and B
// are read identically, so the k positions of both operands agree.
typedef int v16i_t __attribute__((ext_vector_type(16)));
__global__ __launch_bounds__(64) void input_gram_kernel(const int8_t* __restrict__ X, int Kp, int F,
                                                        int32_t* G) {
    const int ti = blockIdx.x, tj = blockIdx.y;
    const int l = threadIdx.x;
    const int8_t* xa = X + (size_t)(32 * ti + (l & 31)) * Kp + 8 * (l >> 5);
    const int8_t* xb = X + (size_t)(32 * tj + (l & 31)) * Kp + 8 * (l >> 5);
    v16i_t acc = {};
    for (int k = 0; k < Kp; k += 16) {
        const long a = *(const long*)(xa + k);
        const long b = *(const long*)(xb + k);
        acc = __builtin_amdgcn_mfma_i32_32x32x16_i8(a, b, acc, 0, 0, 0);
    }
    // Accumulator r of lane l: row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
    const int j = 32 * tj + (l & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 32 * ti + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
        G[(size_t)i * F + j] = acc[r];
    }
}

// Block a: candidates (a, b, s) with b > a (row_n[a]); each also counts for
// its second variable (col_n[b], atomically).
__global__ __launch_bounds__(kInputBlock) void input_count_kernel(PairSource src, int32_t* row_n,
                                                                  int32_t* col_n) {
    const int a = blockIdx.x;
    int local = 0;
    for (int b = a + 1 + (int)threadIdx.x; b < src.n_x; b += kInputBlock) {
        const int2 c = src.counts(a, b);
        const int n = (c.x >= 2) + (c.y >= 2);
        local += n;
        if (n) atomicAdd(&col_n[b], n);
    }
    int total;
    (void)block_exclusive_scan(local, &total);
    if (threadIdx.x == 0) row_n[a] = total;
}

// Exclusive offsets of row_n and col_n (n entries each); out_m = the total.
__global__ __launch_bounds__(kInputBlock) void input_scan_kernel(const int32_t* row_n, const int32_t* col_n,
                                                                 int n, int32_t* row_off, int32_t* col_off,
                                                                 int32_t* out_m) {
    int carry_r = 0, carry_c = 0;
    for (int base = 0; base < n; base += kInputBlock) {
        const int i = base + (int)threadIdx.x;
        int tr, tc;
        const int er = block_exclusive_scan(i < n ? row_n[i] : 0, &tr);
        const int ec = block_exclusive_scan(i < n ? col_n[i] : 0, &tc);
        if (i < n) {
            row_off[i] = carry_r + er;
            col_off[i] = carry_c + ec;
        }
        carry_r += tr;
        carry_c += tc;
    }
    if (threadIdx.x == 0) {
        row_off[n] = carry_r;
        col_off[n] = carry_c;
        out_m[0] = carry_r;
        out_m[1] = carry_c;
    }
}

// Block a: its candidates in key order, (a+1) << 16 | (b+1) << 1 | s with
// '+' before '-', and c in bits 32..41.
__global__ __launch_bounds__(kInputBlock) void input_rows_kernel(PairSource src, const int32_t* row_off,
                                                                 uint64_t* cand) {
    const int a = blockIdx.x;
    int carry = row_off[a];
    const int n_x = src.n_x;
    for (int b0 = a + 1; b0 < n_x; b0 += kInputBlock) {
        const int b = b0 + (int)threadIdx.x;
        int2 c = make_int2(0, 0);
        if (b < n_x) c = src.counts(a, b);
        const bool hp = c.x >= 2, hm = c.y >= 2;
        int total;
        const int pos = carry + block_exclusive_scan(hp + hm, &total);
        const uint64_t key = ((uint64_t)(a + 1) << 16) | ((uint64_t)(b + 1) << 1);
        if (hp) cand[pos] = key | ((uint64_t)c.x << 32);
        if (hm) cand[pos + hp] = key | 1ull | ((uint64_t)c.y << 32);
        carry += total;
    }
}

// Block b: the candidates (x, b, s), x < b, in (x, s) order, as indices into
// the canonical list (found by binary search within x's range).
__global__ __launch_bounds__(kInputBlock) void input_cols_kernel(PairSource src, const int32_t* row_off,
                                                                 const int32_t* col_off, const uint64_t* cand,
                                                                 uint32_t* tl) {
    const int b = blockIdx.x;
    int carry = col_off[b];
    for (int x0 = 0; x0 < b; x0 += kInputBlock) {
        const int x = x0 + (int)threadIdx.x;
        int2 c = make_int2(0, 0);
        if (x < b) c = src.counts(x, b);
        const bool hp = c.x >= 2, hm = c.y >= 2;
        int total;
        const int pos = carry + block_exclusive_scan(hp + hm, &total);
        for (int s = 0; s < 2; ++s) {
            if (!(s ? hm : hp)) continue;
            const uint32_t key = ((uint32_t)(x + 1) << 16) | ((uint32_t)(b + 1) << 1) | (uint32_t)s;
            int lo = row_off[x], hi = row_off[x + 1];
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((uint32_t)cand[mid] < key) lo = mid + 1; else hi = mid;
            }
            tl[pos + (s && hp ? 1 : 0)] = (uint32_t)lo;
        }
        carry += total;
    }
}

}  // namespace csek
