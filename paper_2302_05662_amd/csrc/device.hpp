// Device helpers shared by the SpMV kernels and the batched launcher: aligned
// vector loads of the streamed arrays, the y update and the CSR row body.
#pragma once

#include "common.hpp"

namespace spmv {

typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// ---- N consecutive elements, loaded with the widest aligned vector ----------------

template <class T, int N> struct Pack { T v[N]; };

template <int N>
__device__ __forceinline__ Pack<int32_t, N> ld_i32(const int32_t *p) {
    Pack<int32_t, N> r;
    if constexpr (N == 1) {
        r.v[0] = ld_stream(p);
    } else if constexpr (N == 2) {
        i32x2 a = __builtin_nontemporal_load((const i32x2 *)p);
        r.v[0] = a.x; r.v[1] = a.y;
    } else {
        static_assert(N % 4 == 0, "");
#pragma unroll
        for (int q = 0; q < N; q += 4) {
            i32x4 a = __builtin_nontemporal_load((const i32x4 *)(p + q));
            r.v[q] = a.x; r.v[q + 1] = a.y; r.v[q + 2] = a.z; r.v[q + 3] = a.w;
        }
    }
    return r;
}

template <int N>
__device__ __forceinline__ Pack<float, N> ld_val(const float *p) {
    Pack<float, N> r;
    if constexpr (N == 1) {
        r.v[0] = ld_stream(p);
    } else if constexpr (N == 2) {
        f32x2 a = __builtin_nontemporal_load((const f32x2 *)p);
        r.v[0] = a.x; r.v[1] = a.y;
    } else {
        static_assert(N % 4 == 0, "");
#pragma unroll
        for (int q = 0; q < N; q += 4) {
            f32x4 a = __builtin_nontemporal_load((const f32x4 *)(p + q));
            r.v[q] = a.x; r.v[q + 1] = a.y; r.v[q + 2] = a.z; r.v[q + 3] = a.w;
        }
    }
    return r;
}

template <int N>
__device__ __forceinline__ Pack<double, N> ld_val(const double *p) {
    Pack<double, N> r;
    if constexpr (N == 1) {
        r.v[0] = ld_stream(p);
    } else {
        static_assert(N % 2 == 0, "");
#pragma unroll
        for (int q = 0; q < N; q += 2) {
            f64x2 a = __builtin_nontemporal_load((const f64x2 *)(p + q));
            r.v[q] = a.x; r.v[q + 1] = a.y;
        }
    }
    return r;
}

// N consecutive x values (a cached load, x is reused): vector loads of up to 16
// bytes when p is aligned to them, element loads otherwise.
template <class V, int N>
__device__ __forceinline__ Pack<V, N> ld_xrun(const V *p) {
    Pack<V, N> r;
    constexpr int W = (N * (int)sizeof(V) >= 16) ? 16 / (int)sizeof(V) : N;  // values per load
    if (((uintptr_t)p % (W * sizeof(V))) == 0) {
#pragma unroll
        for (int q = 0; q < N; q += W) {
            if constexpr (W == 4) {
                const f32x4 a = *(const f32x4 *)(p + q);
                r.v[q] = a.x; r.v[q + 1] = a.y; r.v[q + 2] = a.z; r.v[q + 3] = a.w;
            } else if constexpr (W == 2 && sizeof(V) == 8) {
                const f64x2 a = *(const f64x2 *)(p + q);
                r.v[q] = a.x; r.v[q + 1] = a.y;
            } else if constexpr (W == 2) {
                const f32x2 a = *(const f32x2 *)(p + q);
                r.v[q] = a.x; r.v[q + 1] = a.y;
            } else {
#pragma unroll
                for (int j = 0; j < W; ++j) r.v[q + j] = p[q + j];
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j) r.v[j] = p[j];
    }
    return r;
}

// ---- x values of N entries that may be consecutive columns -------------------------
//
// A lane holding N entries whose columns are c, c+1, ..., c+N-1 (banded and
// stencil rows, consecutive ELL rows at one slot) reads them with one vector
// load (dword-aligned: the hardware accepts any 4-byte-aligned address) instead
// of N gathers, so a wave's x instruction touches the few lines of a contiguous
// run rather than N instructions touching the same lines with stride N. Other
// lanes gather each valid entry (masked entries read x[0]). Both paths read the
// same addresses, so the values are identical either way.

typedef float f32x2a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef float f32x4a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef double f64x2a8 __attribute__((ext_vector_type(2), aligned(8)));

template <class V, int N>
__device__ __forceinline__ void ld_x_unaligned(const V *p, V (&xv)[N]) {
    if constexpr (N == 1) {
        xv[0] = p[0];
    } else if constexpr (sizeof(V) == 4 && N == 4) {
        const f32x4a4 a = *(const f32x4a4 *)p;
        xv[0] = a.x; xv[1] = a.y; xv[2] = a.z; xv[3] = a.w;
    } else if constexpr (sizeof(V) == 4 && N == 2) {
        const f32x2a4 a = *(const f32x2a4 *)p;
        xv[0] = a.x; xv[1] = a.y;
    } else {
        static_assert(sizeof(V) == 8 && N % 2 == 0, "");
#pragma unroll
        for (int q = 0; q < N; q += 2) {
            const f64x2a8 a = *(const f64x2a8 *)(p + q);
            xv[q] = a.x; xv[q + 1] = a.y;
        }
    }
}

template <class V, int N>
__device__ __forceinline__ void gather_x(const V *__restrict__ x, const int32_t (&c)[N],
                                         const bool (&ok)[N], V (&xv)[N]) {
    if constexpr (N == 1) {
        xv[0] = x[ok[0] ? c[0] : 0];
        return;
    }
    bool run = ok[0] && ok[N - 1];
#pragma unroll
    for (int q = 1; q < N; ++q) run = run && c[q] == c[0] + q;
    if (run) {
        ld_x_unaligned<V, N>(x + c[0], xv);
    } else {
#pragma unroll
        for (int q = 0; q < N; ++q) xv[q] = x[ok[q] ? c[q] : 0];
    }
}

// y_i = alpha * s + beta * y_i, with y not read when beta == 0.
template <class V>
__device__ __forceinline__ void store_y(V *y, int64_t i, double s, V alpha, V beta) {
    double r = (double)alpha * s;
    if (beta != V(0)) r += (double)beta * (double)y[i];
    y[i] = (V)r;
}

template <int L>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, L);
    return v;
}

// One lane's share of a CSR row's products when NL lanes read 4 consecutive
// entries each per load (aligned 16-byte loads, masked at the row edges).
template <class V, int NL, int UNROLL>
__device__ __forceinline__ double csr_row_partial4(const int32_t *__restrict__ col,
                                                   const V *__restrict__ val,
                                                   const V *__restrict__ x, int32_t s, int32_t e,
                                                   int lane) {
    constexpr int STEP = 4 * NL;
    double acc = 0.0;
    for (int32_t j = (s & ~3) + 4 * lane; j < e; j += STEP * UNROLL) {
        Pack<int32_t, 4> c[UNROLL];
        Pack<V, 4> v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (j + u * STEP < e) {
                c[u] = ld_i32<4>(col + j + u * STEP);
                v[u] = ld_val<4>(val + j + u * STEP);
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            bool ok[4];
            int32_t cc[4];
            V xv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t k = j + u * STEP + q;
                ok[q] = k >= s && k < e;
                cc[q] = c[u].v[q];
            }
            gather_x<V, 4>(x, cc, ok, xv);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (ok[q]) acc += (double)v[u].v[q] * (double)xv[q];
        }
    }
    return acc;
}

// Sum of one CSR row's products by a group of L lanes (L a power of two <= 64).
// Each lane reads 4 consecutive entries per load with an aligned 16-byte load of
// col and of val, starting from the row start rounded down to a multiple of 4;
// entries outside [s, e) are masked before x is read. Arrays are padded to 16
// entries. Every lane of the group returns the same total.
template <class V, int L, int UNROLL>
__device__ __forceinline__ double csr_row_dot4(const int32_t *__restrict__ col,
                                               const V *__restrict__ val,
                                               const V *__restrict__ x, int32_t s, int32_t e,
                                               int lane) {
    return group_sum<L>(csr_row_partial4<V, L, UNROLL>(col, val, x, s, e, lane));
}

// Software-pipelined CSR rows: a group of L lanes walks PASSES rows (row g of
// each pass, bounds in s_rp[p * RPB + g], s_rp[p * RPB + g + 1]) as one stream
// of 4L-entry chunks. Per chunk it issues the x gathers of the current chunk,
// then the col/val loads of the next chunk (the next row's first chunk at a row
// end), and only then accumulates, so HBM latency overlaps gather latency and
// the row reductions. The loop and every state change are wave-uniform (one
// loop while any group of the wave is active, selects instead of branches, an
// empty row counts as one fully masked chunk, the group reduction runs every
// chunk and only its store is conditional), so lane groups never diverge
// around the shuffles.
template <class V, int L, int RPB, int PASSES>
__device__ __forceinline__ void csr_rows_pipelined(const int32_t *__restrict__ col,
                                                   const V *__restrict__ val,
                                                   const V *__restrict__ x,
                                                   const int32_t *s_rp, int g, int lane,
                                                   int64_t row0, int32_t n_rows, V *__restrict__ y,
                                                   V alpha, V beta) {
    constexpr int STEP = 4 * L;
    int p = 0, t = 0;
    int32_t s = s_rp[g], e = s_rp[g + 1];
    int32_t base = s & ~3;
    int32_t chunks = e > s ? (e - base + STEP - 1) / STEP : 1;
    int32_t j = base + 4 * lane;
    // a load address inside the arrays whatever the row: its own chunk, or its start
    Pack<int32_t, 4> c = ld_i32<4>(col + (j < e ? j : base));
    Pack<V, 4> v = ld_val<4>(val + (j < e ? j : base));
    double acc = 0.0;
    bool active = true;
    while (__any(active)) {
        V xv[4];
        bool ok[4];
        int32_t cc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ok[q] = active && (j + q >= s) && (j + q < e);
            cc[q] = c.v[q];
        }
        gather_x<V, 4>(x, cc, ok, xv);
        __builtin_amdgcn_sched_barrier(0);  // gathers issue before the prefetch
        const bool row_done = active && (t + 1 >= chunks);
        const int pn = row_done ? p + 1 : p;
        const bool next_active = active && pn < PASSES;
        const int q_idx = (pn < PASSES ? pn : p) * RPB + g;
        const int32_t sr = s_rp[q_idx], er = s_rp[q_idx + 1];
        const int32_t sn = row_done ? sr : s, en = row_done ? er : e;
        const int32_t basen = sn & ~3;
        const int32_t chunksn = row_done ? (en > sn ? (en - basen + STEP - 1) / STEP : 1) : chunks;
        const int tn = row_done ? 0 : t + 1;
        const int32_t jn = basen + tn * STEP + 4 * lane;
        const int32_t jl = (next_active && jn < en) ? jn : (j < e ? j : base);
        const Pack<int32_t, 4> cn = ld_i32<4>(col + jl);
        const Pack<V, 4> vn = ld_val<4>(val + jl);
        __builtin_amdgcn_sched_barrier(0);  // and the prefetch before the products
        // a select, not a branch: keeps every gather ahead of the prefetch
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double prod = (double)v.v[q] * (double)xv[q];
            acc += ok[q] ? prod : 0.0;
        }
        const double tot = group_sum<L>(acc);
        const int64_t row = row0 + (int64_t)p * RPB + g;
        if (row_done && lane == 0 && row < n_rows) store_y(y, row, tot, alpha, beta);
        acc = row_done ? 0.0 : acc;
        active = next_active;
        p = pn; t = tn; s = sn; e = en; base = basen; chunks = chunksn; j = jn; c = cn; v = vn;
    }
}


// Sum of one sorted block's products into an FP64 accumulator in LDS. The
// block's stream [bs, be) is a whole number of 256-entry chunks in column
// order; inside a chunk the entries are stored transposed, lane l's 16-byte
// group holding entries l, l+64, l+128 and l+192, so one gather instruction
// reads 64 consecutive sorted columns (few distinct cache lines). A step is
// ITEMS/4 consecutive chunks and the NW wavefronts take steps in turn (wave w:
// steps w, w + NW, ...), so the block moves through the columns together and
// the x lines it needs at one time span a narrow window: the blocks on one XCD,
// started together, share that window in its L2. The next step's 16-byte loads
// are in flight during the current step's x gathers. An index packs the row
// inside the block above the low `col_bits` column bits (ROW16: the index is
// the column and the row is the uint16 at the same position of rows16); -1
// marks padding. Loads are clamped to last_load and chunks past be are masked.
// Products are added to s_y[row] with local atomics (no fixed order). Every
// thread calls it.
constexpr int kSortedChunk = 256;

typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

//
// DELTA (column tiles): the packed index holds the column less the first column
// of its chunk, chunk_base[chunk] (chunk = stream position / 256, clamped to
// last_chunk like the loads), so a tall tile's row and column fit 32 bits.
template <class V, int ITEMS, int NW, bool ROW16, bool DELTA = false>
__device__ __forceinline__ void sorted_block_sum(const int32_t *__restrict__ idx,
                                                 const uint16_t *__restrict__ rows16,
                                                 const V *__restrict__ val,
                                                 const V *__restrict__ x, int64_t bs, int64_t be,
                                                 int col_bits, int64_t last_load, double *s_y,
                                                 const int32_t *__restrict__ chunk_base = nullptr,
                                                 int64_t last_chunk = 0) {
    static_assert(ITEMS % 4 == 0, "whole chunks per step");
    constexpr int SUB = ITEMS / 4;
    constexpr int CH = kSortedChunk * SUB;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const uint32_t col_mask = (1u << col_bits) - 1;
    constexpr int64_t STRIDE = (int64_t)CH * NW;
    const int64_t start = bs + (int64_t)CH * w, end = be;
    using CI = Pack<int32_t, 4>;
    using CV = Pack<V, 4>;
    struct Chunk {
        CI c[SUB];
        CV v[SUB];
        u16x4 r[SUB];
        uint32_t base[SUB];
    };
    auto load = [&](int64_t q, Chunk &k) {
#pragma unroll
        for (int u = 0; u < SUB; ++u) {
            const int64_t e = std::min<int64_t>(q + u * kSortedChunk + 4 * lane, last_load);
            k.c[u] = ld_i32<4>(idx + e);
            k.v[u] = ld_val<4>(val + e);
            if constexpr (ROW16) k.r[u] = __builtin_nontemporal_load((const u16x4 *)(rows16 + e));
            if constexpr (DELTA)
                k.base[u] = (uint32_t)chunk_base[std::min<int64_t>((q + u * kSortedChunk) / kSortedChunk,
                                                                   last_chunk)];
        }
    };
    auto step = [&](int64_t q, const Chunk &k, Chunk &kn) {
        V xv[SUB][4];
        bool ok[SUB][4];
#pragma unroll
        for (int u = 0; u < SUB; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                ok[u][j] = (q + u * kSortedChunk < end) && k.c[u].v[j] != -1;
                uint32_t col = ROW16 ? (uint32_t)k.c[u].v[j] : ((uint32_t)k.c[u].v[j] & col_mask);
                if constexpr (DELTA) col += k.base[u];
                xv[u][j] = x[ok[u][j] ? col : 0u];
            }
        __builtin_amdgcn_sched_barrier(0);
        load(q + STRIDE, kn);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < SUB; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (ok[u][j]) {
                    const uint32_t row =
                        ROW16 ? (uint32_t)k.r[u][j] : ((uint32_t)k.c[u].v[j] >> col_bits);
                    atomicAdd(&s_y[row], (double)k.v[u].v[j] * (double)xv[u][j]);
                }
    };
    Chunk kA, kB;
    load(start, kA);
    for (int64_t q = start;;) {  // two steps per pass: the chunk buffers alternate
        if (q >= end) break;
        step(q, kA, kB);
        q += STRIDE;
        if (q >= end) break;
        step(q, kB, kA);
        q += STRIDE;
    }
}

}  // namespace spmv
