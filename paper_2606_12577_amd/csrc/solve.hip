// V-cycle and iterative-refinement solve (gfx950, wave64).
//
// Hot path of every solve:
//   sweep      x_out = x_in - Lambda_l (A x_in - b)     additive, Sec. 2.1
//              x_i  <- x_i - Lambda_{l,k,i} (A x - b)_i  colour k in place, Sec. 2.2
//              reverse applications use Lambda^T in the reversed order, Sec. 2.4
//   residual   r = A x - b, restriction b_c = r_scale P^T r         (Alg. 1)
//   correction x <- x - P x_c                                          (Alg. 1)
//   bottom     x_c = A_c^{-1} b_c (dense FP64 inverse)                 (Alg. 1)
//   refinement FP64 residual b - A x, x += V r                         (solve)
//
// Layout: vectors are [n][R] (the R right-hand sides of one unknown are
// contiguous), A streams as 64-row sliced ELLPACK so that a wavefront reads one
// coalesced column of a slice per step, and Lambda is [B][nb][nb] row-major; the
// forward sweep reads rows of Lambda_l, the reverse sweep rows of the stored
// transposes.  Block residuals are exchanged through LDS inside a workgroup.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include <hip/hip_ext.h>

#include "cs_internal.h"

namespace cs {

namespace {

constexpr int WG = 256;
constexpr int64_t IR_GRID = 1024;   // workgroup cap of the outer-solver kernels (4 per CU)
constexpr int64_t SMALL_SLICES = 8192;   // below this many 64-row slices a level counts as small

template <typename T, int R>
__device__ __forceinline__ void vload(const T *p, T (&o)[R]) {
    constexpr int BYTES = (int)sizeof(T) * R;
    if constexpr (BYTES % 16 == 0) {
        const uint4 *q = reinterpret_cast<const uint4 *>(p);
#pragma unroll
        for (int k = 0; k < BYTES / 16; ++k) {
            uint4 u = q[k];
            __builtin_memcpy(&o[k * (16 / sizeof(T))], &u, 16);
        }
    } else if constexpr (BYTES == 8) {
        uint2 u = *reinterpret_cast<const uint2 *>(p);
        __builtin_memcpy(&o[0], &u, 8);
    } else {
#pragma unroll
        for (int k = 0; k < R; ++k) o[k] = p[k];
    }
}

template <typename T, int R>
__device__ __forceinline__ void vstore(T *p, const T (&o)[R]) {
    constexpr int BYTES = (int)sizeof(T) * R;
    if constexpr (BYTES % 16 == 0) {
        uint4 *q = reinterpret_cast<uint4 *>(p);
#pragma unroll
        for (int k = 0; k < BYTES / 16; ++k) {
            uint4 u;
            __builtin_memcpy(&u, &o[k * (16 / sizeof(T))], 16);
            q[k] = u;
        }
    } else if constexpr (BYTES == 8) {
        uint2 u;
        __builtin_memcpy(&u, &o[0], 8);
        *reinterpret_cast<uint2 *>(p) = u;
    } else {
#pragma unroll
        for (int k = 0; k < R; ++k) p[k] = o[k];
    }
}

// Tiles (256 rows each) handled by this workgroup.  With a workgroup per tile
// the hardware id is remapped by xcd_tile; with fewer workgroups (a multiple
// of 8, resident all at once) each XCD sweeps one contiguous range of tiles
// with its workgroups interleaved, so they advance through the range together.
struct Tiles {
    int64_t t, end, step;
};
__device__ __forceinline__ Tiles my_tiles(int64_t ntiles) {
    const int64_t G = gridDim.x, b = blockIdx.x;
    if (G >= ntiles) return Tiles{xcd_tile(b, G), ntiles, G};
    const int64_t xcd = b & 7, j = b >> 3, gx = G >> 3;
    return Tiles{ntiles * xcd / 8 + j, ntiles * (xcd + 1) / 8, gx};
}

// Loads of the per-sweep streams that are read once (Lambda, b).  FP32 data
// goes through streaming (non-temporal) loads, so that the caches keep the
// gathered x and the matrix: FP32 matrix entries (column, value) are loaded
// normally, every sweep of a level reads the same A, which then stays in the
// 256 MB last-level cache between sweeps (128^3 interface sweep 74.8 -> 70.5
// us; ordinary loads of Lambda and b as well: 76-79 us).  FP64 streams use
// ordinary loads: measured on the 128^3 problem, the FP64 sweep with 8
// right-hand sides takes 173 instead of 202 us, with one 66 instead of 87 us,
// and the FP64 refinement residual 89 instead of 94 us.  FP64 matrices keep
// streaming loads (ordinary ones were 2-6% slower: they do not fit beside the
// FP64 vectors).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <typename T, int R>
__device__ __forceinline__ void vload_nt(const T *p, T (&o)[R]) {
    if constexpr (sizeof(T) == 8) {
        vload<T, R>(p, o);
        return;
    }
    constexpr int BYTES = (int)sizeof(T) * R;
    if constexpr (BYTES % 16 == 0) {
        const u32x4 *q = reinterpret_cast<const u32x4 *>(p);
#pragma unroll
        for (int k = 0; k < BYTES / 16; ++k) {
            u32x4 u = __builtin_nontemporal_load(q + k);
            __builtin_memcpy(&o[k * (16 / sizeof(T))], &u, 16);
        }
    } else if constexpr (BYTES == 8) {
        u32x2 u = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
        __builtin_memcpy(&o[0], &u, 8);
    } else {
#pragma unroll
        for (int k = 0; k < R; ++k) o[k] = __builtin_nontemporal_load(p + k);
    }
}

// x_in at unknown j, minus the interpolated coarse correction when PROL:
// x_in[j] - x_c[j / agg_k]  (contiguous unit aggregation; agg_k divides 64, so
// the division is a shift - a 64-bit division per gathered entry would cost
// more than the gather).
template <typename T, int R, bool PROL>
__device__ __forceinline__ void load_x(const T *xin, const T *xc, int agg_k, int64_t j, T (&o)[R]) {
    vload<T, R>(xin + j * R, o);
    if constexpr (PROL) {
        T cv[R];
        vload<T, R>(xc + (j >> __builtin_ctz((unsigned)agg_k)) * R, cv);
#pragma unroll
        for (int k = 0; k < R; ++k) o[k] -= cv[k];
    }
}

// acc += (A x_in)_row for the SELL row at entry offset `off` (lane included)
// with `len` stored entries.  Column indices and values are fetched U at a
// time before the dependent x gathers, so each wavefront keeps 2U loads and
// then U gathers in flight instead of one chain per entry.
// Exactly L entries, straight-line: L index/value loads, then L gathers, then
// the FMAs, so a wavefront has all of them in flight before its first wait.
template <typename T, int R, bool PROL, int L, typename TA>
__device__ __forceinline__ void spmv_fixed(const int32_t *__restrict__ scol, const TA *__restrict__ sval,
                                           int64_t off, const T *xin, const T *xc, int agg_k, T (&acc)[R]) {
    int cc[L];
    TA aa[L];
#pragma unroll
    for (int u = 0; u < L; ++u) {
        if constexpr (sizeof(TA) == 4) {   // FP32 matrices: keep A in the caches (see above)
            cc[u] = scol[off + (int64_t)u * 64];
            aa[u] = sval[off + (int64_t)u * 64];
        } else {
            cc[u] = __builtin_nontemporal_load(scol + off + (int64_t)u * 64);
            aa[u] = __builtin_nontemporal_load(sval + off + (int64_t)u * 64);
        }
    }
    T xv[L][R];
#pragma unroll
    for (int u = 0; u < L; ++u) load_x<T, R, PROL>(xin, xc, agg_k, cc[u], xv[u]);
#pragma unroll
    for (int u = 0; u < L; ++u) {
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] += (T)aa[u] * xv[u][k];
    }
}

// Rows are processed in straight-line chunks of U = 8 entries and a
// fixed-length tail (also for 64-byte FP64 x rows: 4-entry chunks left the
// FP64 refinement residual at 134 instead of 121 us on the 128^3 problem).
template <typename T, int R, bool PROL, typename TA = T>
__device__ __forceinline__ void spmv_row(const int32_t *__restrict__ scol, const TA *__restrict__ sval, int64_t off,
                                         int len, const T *xin, const T *xc, int agg_k, T (&acc)[R]) {
    constexpr int U = 8;
    int e0 = 0;
    for (; e0 + U <= len; e0 += U)
        spmv_fixed<T, R, PROL, U>(scol, sval, off + (int64_t)e0 * 64, xin, xc, agg_k, acc);
    const int64_t o = off + (int64_t)e0 * 64;
    switch (len - e0) {
        case 1: spmv_fixed<T, R, PROL, 1>(scol, sval, o, xin, xc, agg_k, acc); break;
        case 2: spmv_fixed<T, R, PROL, 2>(scol, sval, o, xin, xc, agg_k, acc); break;
        case 3: spmv_fixed<T, R, PROL, 3>(scol, sval, o, xin, xc, agg_k, acc); break;
        case 4: if constexpr (U > 4) spmv_fixed<T, R, PROL, 4>(scol, sval, o, xin, xc, agg_k, acc); break;
        case 5: if constexpr (U > 5) spmv_fixed<T, R, PROL, 5>(scol, sval, o, xin, xc, agg_k, acc); break;
        case 6: if constexpr (U > 6) spmv_fixed<T, R, PROL, 6>(scol, sval, o, xin, xc, agg_k, acc); break;
        case 7: if constexpr (U > 7) spmv_fixed<T, R, PROL, 7>(scol, sval, o, xin, xc, agg_k, acc); break;
        default: break;
    }
}

// One cascade sweep over 4 SELL slices (256 rows) per workgroup.
//   ZERO:   x_in = 0, so x_out = Lambda b (A is not read)
//   ROWMAP: rows come from a colour list and x is updated in place
//   PROL:   x_in is first corrected by the coarse-grid solution x_c (the
//           interpolation step of Alg. 1 fused into the first post-sweep)
//   WGS:    workgroup size; 256 (4 slices) on large levels, 64 (one slice per
//           workgroup, more workgroups in flight) on small ones
// SpMV of a natural-order row of an NB-block level (row = 64 slice + lane, so
// a block's rows sit in NB consecutive lanes and the slice's 64 rows in its 64
// lanes): entries whose column lies in the row's own slice take x from the
// lane that holds that row (a shuffle of the x row every lane loads for its
// own row anyway), only the others are gathered.  With the Morton numbering a
// slice is a 4x4x4 cube of cells, so for the 7-point stencil about 1.5 of the
// 7 entries per row are gathered (3 when only the own 2x2x2 block was served
// this way).  Every active lane of the slice holds its row's x: a valid row
// couples only to valid rows, which run the same code.
template <typename T, int R, bool PROL, int NB, int L>
__device__ __forceinline__ void spmv_fixed_blk(const int32_t *__restrict__ scol, const T *__restrict__ sval,
                                               int64_t off, const T *xin, const T *xc, int agg_k, int64_t row,
                                               int lane, const T (&xo)[R], T (&acc)[R]) {
    int cc[L];
    T aa[L];
#pragma unroll
    for (int u = 0; u < L; ++u) {
        if constexpr (sizeof(T) == 4) {   // FP32 matrices: keep A in the caches (see above)
            cc[u] = scol[off + (int64_t)u * 64];
            aa[u] = sval[off + (int64_t)u * 64];
        } else {
            cc[u] = __builtin_nontemporal_load(scol + off + (int64_t)u * 64);
            aa[u] = __builtin_nontemporal_load(sval + off + (int64_t)u * 64);
        }
    }
    const int64_t first = row - lane;   // the slice's first row
    T xv[L][R];
#pragma unroll
    for (int u = 0; u < L; ++u) {
        const int64_t d = (int64_t)cc[u] - first;
        const int src = (int)(d & 63);
#pragma unroll
        for (int k = 0; k < R; ++k) xv[u][k] = __shfl(xo[k], src, 64);
        if (d < 0 || d >= 64) load_x<T, R, PROL>(xin, xc, agg_k, cc[u], xv[u]);
    }
#pragma unroll
    for (int u = 0; u < L; ++u) {
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] += aa[u] * xv[u][k];
    }
}

template <typename T, int R, bool PROL, int NB>
__device__ __forceinline__ void spmv_row_blk(const int32_t *__restrict__ scol, const T *__restrict__ sval,
                                             int64_t off, int len, const T *xin, const T *xc, int agg_k,
                                             int64_t row, int lane, const T (&xo)[R], T (&acc)[R]) {
    constexpr int U = 8;
    int e0 = 0;
    for (; e0 + U <= len; e0 += U)
        spmv_fixed_blk<T, R, PROL, NB, U>(scol, sval, off + (int64_t)e0 * 64, xin, xc, agg_k, row, lane, xo, acc);
    const int64_t o = off + (int64_t)e0 * 64;
    switch (len - e0) {
        case 1: spmv_fixed_blk<T, R, PROL, NB, 1>(scol, sval, o, xin, xc, agg_k, row, lane, xo, acc); break;
        case 2: spmv_fixed_blk<T, R, PROL, NB, 2>(scol, sval, o, xin, xc, agg_k, row, lane, xo, acc); break;
        case 3: spmv_fixed_blk<T, R, PROL, NB, 3>(scol, sval, o, xin, xc, agg_k, row, lane, xo, acc); break;
        case 4: if constexpr (U > 4) spmv_fixed_blk<T, R, PROL, NB, 4>(scol, sval, o, xin, xc, agg_k, row, lane, xo, acc); break;
        case 5: if constexpr (U > 5) spmv_fixed_blk<T, R, PROL, NB, 5>(scol, sval, o, xin, xc, agg_k, row, lane, xo, acc); break;
        case 6: if constexpr (U > 6) spmv_fixed_blk<T, R, PROL, NB, 6>(scol, sval, o, xin, xc, agg_k, row, lane, xo, acc); break;
        case 7: if constexpr (U > 7) spmv_fixed_blk<T, R, PROL, NB, 7>(scol, sval, o, xin, xc, agg_k, row, lane, xo, acc); break;
        default: break;
    }
}

// Natural-order SpMV row of a level with NB-blocks: the in-block shuffle form
// (xo: the row's own x, already loaded) where it pays, i.e. for blocks of at
// most 8 rows and gathered rows of at least 16 bytes (every entry costs the
// shuffles of a whole x row, a saved gather only for in-block entries: with
// one FP64 right-hand side, or 16 x 16 blocks, plain gathers measured faster).
template <typename T, int R, bool PROL, int NB>
__device__ __forceinline__ void spmv_row_nb(const int32_t *__restrict__ scol, const T *__restrict__ sval, int64_t off,
                                            int len, const T *xin, const T *xc, int agg_k, int64_t row, int lane,
                                            const T (&xo)[R], T (&acc)[R]) {
    if constexpr (NB > 1 && NB <= 8 && sizeof(T) * R >= 16)
        spmv_row_blk<T, R, PROL, NB>(scol, sval, off, len, xin, xc, agg_k, row, lane, xo, acc);
    else
        spmv_row<T, R, PROL>(scol, sval, off, len, xin, xc, agg_k, acc);
}

// The sweep's result for a row: stored as x_out, or with ACC added into the
// FP64 vector acc instead (x_out is not written): the update x += d of an
// outer refinement folded into the V-cycle's last fine-level sweep, with the
// same FP64 addition as a separate pass.
template <typename T, int R, bool ACC>
__device__ __forceinline__ void sweep_store(T *xout, double *acc, int64_t row, const T (&xo)[R]) {
    if constexpr (ACC) {
        double ax[R];
        vload<double, R>(acc + row * R, ax);
#pragma unroll
        for (int k = 0; k < R; ++k) ax[k] += (double)xo[k];
        vstore<double, R>(acc + row * R, ax);
    } else {
        vstore<T, R>(xout + row * R, xo);
    }
}

// One tile (WGS/64 slices) of a cascade sweep; red: LDS of WGS * R values
// (block levels), rewritten per tile.
template <typename T, int NB, int R, bool ZERO, bool ROWMAP, bool PROL, int WGS, bool ACC = false>
__device__ __forceinline__ void sweep_tile(int64_t tile, int64_t nrows, int64_t nslices,
                                           const int32_t *__restrict__ rows, const int64_t *__restrict__ sptr,
                                           const int32_t *__restrict__ slen, const int32_t *__restrict__ scol,
                                           const T *__restrict__ sval, const T *__restrict__ lam,
                                           const T *__restrict__ b, const T *xin, T *xout,
                                           const T *__restrict__ xc, int agg_k, T *red, double *acc = nullptr) {
    constexpr int SPW = WGS / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t slice = tile * SPW + wv;
    const int64_t q = slice * 64 + lane;
    const bool valid = slice < nslices && q < nrows;
    int64_t row = 0;
    if (valid) row = ROWMAP ? (int64_t)rows[q] : q;
    T res[R];
#pragma unroll
    for (int k = 0; k < R; ++k) res[k] = T(0);
    // block levels: the row of Lambda and the row's own x_in are loaded first;
    // x_in feeds the in-slice part of the SpMV through lane shuffles
    T lr[NB], xo[R];
    if constexpr (NB > 1) {
        if (valid) {
            vload_nt<T, NB>(lam + (row / NB) * (NB * NB) + (lane % NB) * NB, lr);
            if constexpr (ZERO) {
#pragma unroll
                for (int k = 0; k < R; ++k) xo[k] = T(0);
            } else {
                load_x<T, R, PROL>(xin, xc, agg_k, row, xo);
            }
        }
    }
    if (valid) {
        T bb[R];
        vload_nt<T, R>(b + row * R, bb);
#pragma unroll
        for (int k = 0; k < R; ++k) res[k] = -bb[k];
        if constexpr (!ZERO) {
            if constexpr (NB > 1 && NB <= 8 && !ROWMAP && sizeof(T) * R >= 16)
                spmv_row_blk<T, R, PROL, NB>(scol, sval, sptr[slice] + lane, slen[slice], xin, xc, agg_k, row,
                                             lane, xo, res);
            else
                spmv_row<T, R, PROL>(scol, sval, sptr[slice] + lane, slen[slice], xin, xc, agg_k, res);
        }
    }
    if constexpr (NB == 1) {
        if (valid) {
            const T l = __builtin_nontemporal_load(lam + row);
            T xo[R];
            if constexpr (ZERO) {
#pragma unroll
                for (int k = 0; k < R; ++k) xo[k] = T(0);
            } else {
                load_x<T, R, PROL>(xin, xc, agg_k, row, xo);
            }
#pragma unroll
            for (int k = 0; k < R; ++k) xo[k] -= l * res[k];
            sweep_store<T, R, ACC>(xout, acc, row, xo);
        }
    } else {
#pragma unroll
        for (int k = 0; k < R; ++k) red[threadIdx.x * R + k] = res[k];
        __syncthreads();
        if (valid) {
            const int rloc = lane % NB;
            const int base = threadIdx.x - rloc;
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) {
#pragma unroll
                for (int k = 0; k < R; ++k) xo[k] -= lr[cc] * red[(base + cc) * R + k];
            }
            sweep_store<T, R, ACC>(xout, acc, row, xo);
        }
        __syncthreads();   // red is rewritten by the next tile
    }
}

template <typename T, int NB, int R, bool ZERO, bool ROWMAP, bool PROL, int WGS, bool ACC = false>
__global__ __launch_bounds__(WGS) void k_sweep(int64_t nrows, int64_t nslices, const int32_t *__restrict__ rows,
                                               const int64_t *__restrict__ sptr, const int32_t *__restrict__ slen,
                                               const int32_t *__restrict__ scol, const T *__restrict__ sval,
                                               const T *__restrict__ lam, const T *__restrict__ b, const T *xin,
                                               T *xout, const T *__restrict__ xc, int agg_k, double *acc) {
    constexpr int SPW = WGS / 64;
    __shared__ T red[NB > 1 ? WGS * R : 1];
    const Tiles tl = my_tiles((nslices + SPW - 1) / SPW);
    for (int64_t tile = tl.t; tile < tl.end; tile += tl.step)
        sweep_tile<T, NB, R, ZERO, ROWMAP, PROL, WGS, ACC>(tile, nrows, nslices, rows, sptr, slen, scol, sval, lam,
                                                           b, xin, xout, xc, agg_k, red, acc);
}

// r = A x - b over SELL rows (natural order)
template <typename T, int R>
__global__ __launch_bounds__(WG) void k_residual(int64_t nrows, int64_t nslices, const int64_t *__restrict__ sptr,
                                                 const int32_t *__restrict__ slen, const int32_t *__restrict__ scol,
                                                 const T *__restrict__ sval, const T *__restrict__ b,
                                                 const T *__restrict__ x, T *__restrict__ r) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const Tiles tl = my_tiles((nslices + 3) / 4);
    for (int64_t tile = tl.t; tile < tl.end; tile += tl.step) {
        const int64_t slice = tile * 4 + wv;
        const int64_t row = slice * 64 + lane;
        if (slice >= nslices || row >= nrows) continue;
        T acc[R];
        vload_nt<T, R>(b + row * R, acc);
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = -acc[k];
        spmv_row<T, R, false>(scol, sval, sptr[slice] + lane, slen[slice], x, nullptr, 1, acc);
        vstore<T, R>(r + row * R, acc);
    }
}

// Fused residual and restriction for contiguous unit aggregation:
// b_c[I] = r_scale * sum_{u < agg_k} (A x - b)[agg_k*I + u].  A tile holds
// WGS fine rows, i.e. WGS/agg_k whole coarse rows (agg_k divides 64); red:
// LDS of WGS * R values.
template <typename T, int R, int NB, int WGS>
__device__ __forceinline__ void residual_restrict_tile(int64_t tile, int64_t nrows, int64_t nslices,
                                                       const int64_t *__restrict__ sptr,
                                                       const int32_t *__restrict__ slen,
                                                       const int32_t *__restrict__ scol,
                                                       const T *__restrict__ sval, const T *__restrict__ b,
                                                       const T *__restrict__ x, int agg_k, int64_t nc, T r_scale,
                                                       T *__restrict__ bc, T *red) {
    constexpr int SPW = WGS / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t slice = tile * SPW + wv;
    const int64_t row = slice * 64 + lane;
    T acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = T(0);
    if (slice < nslices && row < nrows) {
        T xo[R];
        if constexpr (NB > 1) vload<T, R>(x + row * R, xo);
        vload_nt<T, R>(b + row * R, acc);
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = -acc[k];
        spmv_row_nb<T, R, false, NB>(scol, sval, sptr[slice] + lane, slen[slice], x, nullptr, 1, row, lane, xo, acc);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) red[threadIdx.x * R + k] = acc[k];
    __syncthreads();
    const int per = WGS / agg_k;
    if ((int)threadIdx.x < per) {
        const int64_t I = tile * per + threadIdx.x;
        if (I < nc) {
            T s[R];
#pragma unroll
            for (int k = 0; k < R; ++k) s[k] = T(0);
            for (int u = 0; u < agg_k; ++u) {
#pragma unroll
                for (int k = 0; k < R; ++k) s[k] += red[(threadIdx.x * agg_k + u) * R + k];
            }
#pragma unroll
            for (int k = 0; k < R; ++k) s[k] *= r_scale;
            vstore<T, R>(bc + I * R, s);
        }
    }
    __syncthreads();   // red is rewritten by the next tile
}

template <typename T, int R, int NB = 1>
__global__ __launch_bounds__(WG) void k_residual_restrict(int64_t nrows, int64_t nslices,
                                                          const int64_t *__restrict__ sptr,
                                                          const int32_t *__restrict__ slen,
                                                          const int32_t *__restrict__ scol, const T *__restrict__ sval,
                                                          const T *__restrict__ b, const T *__restrict__ x,
                                                          int agg_k, int64_t nc, T r_scale, T *__restrict__ bc) {
    __shared__ T red[WG * R];
    const Tiles tl = my_tiles((nslices + 3) / 4);
    for (int64_t tile = tl.t; tile < tl.end; tile += tl.step)
        residual_restrict_tile<T, R, NB, WG>(tile, nrows, nslices, sptr, slen, scol, sval, b, x, agg_k, nc, r_scale,
                                             bc, red);
}

// b_c = r_scale * P^T r with P^T in sliced ELLPACK (a lane per coarse row,
// coalesced column/value streams)
template <typename T, int R>
__global__ __launch_bounds__(WG) void k_restrict_sell(int64_t nc, int64_t nslices, const int64_t *__restrict__ sptr,
                                                      const int32_t *__restrict__ slen,
                                                      const int32_t *__restrict__ scol, const T *__restrict__ sval,
                                                      T r_scale, const T *__restrict__ r, T *__restrict__ bc) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const Tiles tl = my_tiles((nslices + 3) / 4);
    for (int64_t tile = tl.t; tile < tl.end; tile += tl.step) {
        const int64_t slice = tile * 4 + wv;
        const int64_t row = slice * 64 + lane;
        if (slice >= nslices || row >= nc) continue;
        T acc[R];
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = T(0);
        spmv_row<T, R, false>(scol, sval, sptr[slice] + lane, slen[slice], r, nullptr, 1, acc);
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] *= r_scale;
        vstore<T, R>(bc + row * R, acc);
    }
}

// x <- x - P x_c with P in sliced ELLPACK, rows [0, n)
template <typename T, int R>
__global__ __launch_bounds__(WG) void k_prolong_sell(int64_t n, int64_t nslices, const int64_t *__restrict__ sptr,
                                                     const int32_t *__restrict__ slen,
                                                     const int32_t *__restrict__ scol, const T *__restrict__ sval,
                                                     const T *__restrict__ xc, T *__restrict__ x) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const Tiles tl = my_tiles((nslices + 3) / 4);
    for (int64_t tile = tl.t; tile < tl.end; tile += tl.step) {
        const int64_t slice = tile * 4 + wv;
        const int64_t row = slice * 64 + lane;
        if (slice >= nslices || row >= n) continue;
        T acc[R];
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = T(0);
        spmv_row<T, R, false>(scol, sval, sptr[slice] + lane, slen[slice], xc, nullptr, 1, acc);
        T xo[R];
        vload<T, R>(x + row * R, xo);
#pragma unroll
        for (int k = 0; k < R; ++k) xo[k] -= acc[k];
        vstore<T, R>(x + row * R, xo);
    }
}


// Direct segments: x[i] = sum_j inv_q[i - s_q][j] b[s_q + j] for the rows
// [n_active, n), with inv_q the FP64 inverse of the diagonal block of segment q
// (the whole bottom level, or trailing systems of a batch that end on this
// level).  One wavefront per row: the lanes stream the inverse row coalesced,
// accumulate all right-hand sides in FP64 and reduce across the wavefront.
// Row i of a direct segment: x_i = (A_seg^{-1} b_seg)_i with FP64
// accumulation, one wavefront per row.
template <typename T, int R>
__device__ __forceinline__ void direct_row(int64_t i, int nseg, const int64_t *__restrict__ seg,
                                           const int64_t *__restrict__ inv_off, const double *__restrict__ inv,
                                           const T *__restrict__ b, T *__restrict__ x) {
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = nseg - 1;   // segment q with seg[q] <= i < seg[q+1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    const int64_t s = seg[lo], m = seg[lo + 1] - s;
    const double *row = inv + inv_off[lo] + (i - s) * m;
    double acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = 0.0;
    for (int64_t j = lane; j < m; j += 64) {
        const double a = row[j];
        T bv[R];
        vload<T, R>(b + (s + j) * R, bv);
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] += a * (double)bv[k];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] += __shfl_xor(acc[k], off, 64);
    }
    if (lane == 0) {
        T o[R];
#pragma unroll
        for (int k = 0; k < R; ++k) o[k] = (T)acc[k];
        vstore<T, R>(x + i * R, o);
    }
}

template <typename T, int R>
__global__ __launch_bounds__(WG) void k_direct_seg(int64_t n_active, int64_t n, int nseg,
                                                   const int64_t *__restrict__ seg, const int64_t *__restrict__ inv_off,
                                                   const double *__restrict__ inv, const T *__restrict__ b,
                                                   T *__restrict__ x) {
    const int64_t i = n_active + (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    if (i >= n) return;   // uniform per wavefront
    direct_row<T, R>(i, nseg, seg, inv_off, inv, b, x);
}

// ---------------------------------------------------------------------------
// Single-workgroup tail V-cycle: the coarse levels of at most a few thousand
// rows are latency-bound (a kernel of a few microseconds per sweep, transfer
// and direct solve), so one workgroup of 512-1024 threads runs Alg. 1 on all of
// them in one launch: the same per-row arithmetic as the per-level kernels
// (sweep_tile, residual_restrict_tile, direct_row), a workgroup barrier where
// the eager path has a kernel boundary, hence identical results.
// ---------------------------------------------------------------------------
// 1024 threads where a row's vector data fits in 8 bytes; 512 (twice the
// registers per thread) for several right-hand sides
template <typename T, int R>
constexpr int tail_wg() { return R * sizeof(T) <= 8 ? 1024 : 512; }

template <typename T, int NB, int R, int TW, bool ZERO, bool PROL>
__device__ void tail_sweep(const TailLevel &L, const T *lam, const T *b, const T *xin, T *xout, const T *xc,
                           T *red) {
    constexpr int SPW = TW / 64;
    const int64_t ntiles = (L.nslices + SPW - 1) / SPW;
    for (int64_t tile = 0; tile < ntiles; ++tile)
        sweep_tile<T, NB, R, ZERO, false, PROL, TW>(tile, L.n_active, L.nslices, nullptr, L.sptr, L.slen, L.scol,
                                                        static_cast<const T *>(L.sval), lam, b, xin, xout, xc,
                                                        L.agg_k, red);
    __syncthreads();
}

// one application of the level's additive cascade (as apply_cascade); returns
// the buffer that holds the result
template <typename T, int NB, int R, int TW>
__device__ T *tail_cascade(const TailLevel &L, bool reverse, bool zero_start, const T *b, T *x, T *alt,
                           const T *xc, T *red) {
    T *cur = x, *nxt = alt;
    for (int s = 0; s < L.depth; ++s) {
        const int ell = reverse ? L.depth - 1 - s : s;
        const T *lam = static_cast<const T *>(reverse ? L.lamT : L.lam) + (int64_t)ell * L.nbl;
        if (zero_start && s == 0) tail_sweep<T, NB, R, TW, true, false>(L, lam, b, cur, nxt, nullptr, red);
        else if (s == 0 && xc) tail_sweep<T, NB, R, TW, false, true>(L, lam, b, cur, nxt, xc, red);
        else tail_sweep<T, NB, R, TW, false, false>(L, lam, b, cur, nxt, nullptr, red);
        T *t = cur;
        cur = nxt;
        nxt = t;
    }
    return cur;
}

template <typename T, int R, int TW>
__device__ void tail_direct(const TailLevel &L, T *x) {
    const int wv = threadIdx.x >> 6;
    for (int64_t i = L.n_active + wv; i < L.n; i += TW / 64)
        direct_row<T, R>(i, L.nseg, L.dseg, L.dinv_off, L.dinv, static_cast<const T *>(L.bb), x);
    __syncthreads();
}

// Alg. 1 from tab[0] (its right-hand side already in tab[0].bb) to the last
// entry, solved directly; the result in tab[0].xb.
template <typename T, int NB, int R, int TW = tail_wg<T, R>()>
__global__ __launch_bounds__(TW) void k_tail_vcycle(const TailLevel *__restrict__ tab, int nlev, int n_pre,
                                                    int n_post, int rf) {
    __shared__ T red[TW * R];
    uint32_t in_alt = 0;   // bit l: level l's smoothed x sits in xt instead of xb
    for (int l = 0; l + 1 < nlev; ++l) {
        const TailLevel &L = tab[l];
        T *x = static_cast<T *>(L.xb), *alt = static_cast<T *>(L.xt);
        const T *b = static_cast<const T *>(L.bb);
        for (int a = 0; a < n_pre; ++a) {
            T *res = tail_cascade<T, NB, R, TW>(L, rf != 0, a == 0, b, x, alt, nullptr, red);
            if (res != x) {
                alt = x;
                x = res;
            }
        }
        if (x != static_cast<T *>(L.xb)) in_alt |= 1u << l;
        constexpr int SPW = TW / 64;
        const int64_t ntiles = (L.nslices + SPW - 1) / SPW;
        for (int64_t tile = 0; tile < ntiles; ++tile)
            residual_restrict_tile<T, R, NB, TW>(tile, L.n_active, L.nslices, L.sptr, L.slen, L.scol,
                                                     static_cast<const T *>(L.sval), b, x, L.agg_k, L.nc,
                                                     (T)L.r_scale, static_cast<T *>(tab[l + 1].bb), red);
        __syncthreads();
    }
    tail_direct<T, R, TW>(tab[nlev - 1], static_cast<T *>(tab[nlev - 1].xb));
    for (int l = nlev - 2; l >= 0; --l) {
        const TailLevel &L = tab[l];
        T *xb = static_cast<T *>(L.xb), *xt = static_cast<T *>(L.xt);
        T *x = (in_alt >> l) & 1u ? xt : xb, *alt = x == xb ? xt : xb;
        const T *b = static_cast<const T *>(L.bb);
        const T *xc = static_cast<const T *>(tab[l + 1].xb);
        for (int a = 0; a < n_post; ++a) {
            T *res = tail_cascade<T, NB, R, TW>(L, false, false, b, x, alt, a == 0 ? xc : nullptr, red);
            if (res != x) {
                alt = x;
                x = res;
            }
        }
        if (x != xb) {
            for (int64_t e = threadIdx.x; e < L.n_active * R; e += TW) xb[e] = x[e];
            __syncthreads();
        }
        tail_direct<T, R, TW>(L, xb);
    }
}

// Per-workgroup sums of W per-thread values into partial[blockIdx.x][W] (red:
// (WG / 64) * W doubles): a wavefront butterfly, then the waves in order.
template <int W>
__device__ __forceinline__ void wg_partials(const double (&acc)[W], double *red, double *partial) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wv * W + k] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < W) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < WG / 64; ++w) t += red[w * W + threadIdx.x];
        partial[(int64_t)blockIdx.x * W + threadIdx.x] = t;
    }
}

// FP64 refinement residual r = b - A x; writes r in the working precision and
// per-workgroup partial sums of r^2 for every right-hand side.  With x == null
// it computes the partial sums of b^2.
//
// SYS (a batch of independent systems): the squares are summed per 64-row
// slice instead.  het[s] < 0 marks a slice whose rows all belong to one
// system: its sums go to spart[s][R] (wavefront reduction).  The few slices
// that straddle a system boundary keep their per-row squares in
// rn2[(het[s]*64 + lane)][R] for the per-system reduction.
template <typename T, int R, bool SYS, int NB = 1>
__global__ __launch_bounds__(WG) void k_ir_residual(int64_t nrows, int64_t nslices, const int64_t *__restrict__ sptr,
                                                    const int32_t *__restrict__ slen, const int32_t *__restrict__ scol,
                                                    const double *__restrict__ sval, const double *__restrict__ b,
                                                    const double *__restrict__ x, T *__restrict__ rt,
                                                    double *__restrict__ partial, const int32_t *__restrict__ het,
                                                    double *__restrict__ spart, double *__restrict__ rn2) {
    __shared__ double red[SYS ? 1 : (WG / 64) * R];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t ntiles = (nslices + 3) / 4;
    double sq[R];
#pragma unroll
    for (int k = 0; k < R; ++k) sq[k] = 0.0;
    // grid-stride over 256-row tiles; partial sums stay in registers
    const Tiles tl = my_tiles(ntiles);
    for (int64_t tile = tl.t; tile < tl.end; tile += tl.step) {
        const int64_t slice = tile * 4 + wv;
        const int64_t row = slice * 64 + lane;
        if (slice >= nslices) continue;   // uniform per wavefront
        const bool valid = row < nrows;
        if (!SYS && !valid) continue;
        double acc[R];
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = 0.0;
        if (valid) {
            vload_nt<double, R>(b + row * R, acc);
            if (x) {
                double ax[R], xo[R];
#pragma unroll
                for (int k = 0; k < R; ++k) ax[k] = 0.0;
                if constexpr (NB > 1) vload<double, R>(x + row * R, xo);
                spmv_row_nb<double, R, false, NB>(scol, sval, sptr[slice] + lane, slen[slice], x, nullptr, 1, row,
                                                  lane, xo, ax);
#pragma unroll
                for (int k = 0; k < R; ++k) acc[k] -= ax[k];
            }
            if (rt) {
                T o[R];
#pragma unroll
                for (int k = 0; k < R; ++k) o[k] = (T)acc[k];
                vstore<T, R>(rt + row * R, o);
            }
        }
        if constexpr (SYS) {
            double o[R];
#pragma unroll
            for (int k = 0; k < R; ++k) o[k] = acc[k] * acc[k];
            const int h = het[slice];
            if (h < 0) {
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
                    for (int k = 0; k < R; ++k) o[k] += __shfl_xor(o[k], off, 64);
                }
                if (lane == 0) vstore<double, R>(spart + slice * R, o);
            } else {
                vstore<double, R>(rn2 + ((int64_t)h * 64 + lane) * R, o);
            }
        } else {
#pragma unroll
            for (int k = 0; k < R; ++k) sq[k] += acc[k] * acc[k];
        }
    }
    if constexpr (SYS) return;
    else wg_partials<R>(sq, red, partial);
}

// ---------------------------------------------------------------------------
// Flexible conjugate gradients around the V-cycle (FP64 outer vectors)
// ---------------------------------------------------------------------------

// Partial sums of W per-row values: per 64-row slice (SYS, see k_ir_residual)
// or accumulated per thread for a workgroup tree (acc).
template <int W>
__device__ __forceinline__ void slice_partials(double (&v)[W], int lane, int64_t slice, const int32_t *het,
                                               double *spart, double *rn2) {
    const int h = het[slice];
    if (h < 0) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int k = 0; k < W; ++k) v[k] += __shfl_xor(v[k], off, 64);
        }
        if (lane == 0) vstore<double, W>(spart + slice * W, v);
    } else {
        vstore<double, W>(rn2 + ((int64_t)h * 64 + lane) * W, v);
    }
}


__device__ __forceinline__ int row_system(int64_t row, int nsys, const int64_t *__restrict__ sys_ptr) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sys_ptr[mid] <= row) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// (z, q) per right-hand side
template <typename T, int R, bool SYS>
__global__ __launch_bounds__(WG) void k_cg_zq(int64_t nrows, int64_t nslices, const T *__restrict__ z,
                                              const double *__restrict__ q, const int32_t *__restrict__ het,
                                              double *__restrict__ spart, double *__restrict__ rn2,
                                              double *__restrict__ partial) {
    __shared__ double red[SYS ? 1 : (WG / 64) * R];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = 0.0;
    const Tiles tl = my_tiles((nslices + 3) / 4);
    for (int64_t tile = tl.t; tile < tl.end; tile += tl.step) {
        const int64_t slice = tile * 4 + wv;
        if (slice >= nslices) continue;
        const int64_t row = slice * 64 + lane;
        double v[R];
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = 0.0;
        if (row < nrows) {
            T zz[R];
            double qq[R];
            vload_nt<T, R>(z + row * R, zz);
            vload_nt<double, R>(q + row * R, qq);
#pragma unroll
            for (int k = 0; k < R; ++k) v[k] = (double)zz[k] * qq[k];
        }
        if constexpr (SYS) {
            slice_partials<R>(v, lane, slice, het, spart, rn2);
        } else {
#pragma unroll
            for (int k = 0; k < R; ++k) acc[k] += v[k];
        }
    }
    if constexpr (!SYS) wg_partials<R>(acc, red, partial);
}

// p = z + beta p with beta = -(z, q_prev) / (p_prev, q_prev) per system and
// right-hand side (first: p = z).  pq_prev holds [nsys][2R]: (p, q) then (p, r).
template <typename T, int R>
__global__ void k_cg_p(int64_t n, int nsys, const int64_t *__restrict__ sys_ptr, const T *__restrict__ z,
                       const double *__restrict__ zq, const double *__restrict__ pq_prev, double *__restrict__ p,
                       int first) {
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row >= n) return;
    const int s = nsys > 1 ? row_system(row, nsys, sys_ptr) : 0;
    T zz[R];
    double pp[R];
    vload<T, R>(z + row * R, zz);
    if (!first) vload<double, R>(p + row * R, pp);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        double beta = 0.0;
        if (!first) {
            const double d = pq_prev[s * 2 * R + k];
            beta = d > 0.0 ? -zq[s * R + k] / d : 0.0;
            if (!isfinite(beta)) beta = 0.0;
        }
        pp[k] = (double)zz[k] + (first ? 0.0 : beta * pp[k]);
    }
    vstore<double, R>(p + row * R, pp);
}

// q = A p (FP64) with the per-RHS partial sums of (p, q) and (p, r)
template <int R, bool SYS, int NB = 1>
__global__ __launch_bounds__(WG) void k_cg_ap(int64_t nrows, int64_t nslices, const int64_t *__restrict__ sptr,
                                              const int32_t *__restrict__ slen, const int32_t *__restrict__ scol,
                                              const double *__restrict__ sval, const double *__restrict__ p,
                                              const double *__restrict__ r, double *__restrict__ q,
                                              const int32_t *__restrict__ het, double *__restrict__ spart,
                                              double *__restrict__ rn2, double *__restrict__ partial) {
    __shared__ double red[SYS ? 1 : (WG / 64) * 2 * R];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double acc[2 * R];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) acc[k] = 0.0;
    const Tiles tl = my_tiles((nslices + 3) / 4);
    for (int64_t tile = tl.t; tile < tl.end; tile += tl.step) {
        const int64_t slice = tile * 4 + wv;
        if (slice >= nslices) continue;
        const int64_t row = slice * 64 + lane;
        double v[2 * R];
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) v[k] = 0.0;
        if (row < nrows) {
            double ap[R], pp[R], rr[R];
#pragma unroll
            for (int k = 0; k < R; ++k) ap[k] = 0.0;
            vload<double, R>(p + row * R, pp);
            spmv_row_nb<double, R, false, NB>(scol, sval, sptr[slice] + lane, slen[slice], p, nullptr, 1, row, lane,
                                              pp, ap);
            vstore<double, R>(q + row * R, ap);
            vload_nt<double, R>(r + row * R, rr);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                v[k] = pp[k] * ap[k];
                v[R + k] = pp[k] * rr[k];
            }
        }
        if constexpr (SYS) {
            slice_partials<2 * R>(v, lane, slice, het, spart, rn2);
        } else {
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) acc[k] += v[k];
        }
    }
    if constexpr (!SYS) wg_partials<2 * R>(acc, red, partial);
}

// x += alpha p, r -= alpha q with alpha = (p, r) / (p, q); rt = r in the
// working precision; per-RHS partial sums of r^2
template <typename T, int R, bool SYS>
__global__ __launch_bounds__(WG) void k_cg_update(int64_t nrows, int64_t nslices, int nsys,
                                                  const int64_t *__restrict__ sys_ptr, const double *__restrict__ pq,
                                                  const double *__restrict__ p, const double *__restrict__ q,
                                                  double *__restrict__ x, double *__restrict__ r, T *__restrict__ rt,
                                                  const int32_t *__restrict__ het, double *__restrict__ spart,
                                                  double *__restrict__ rn2, double *__restrict__ partial) {
    __shared__ double red[SYS ? 1 : (WG / 64) * R];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = 0.0;
    const Tiles tl = my_tiles((nslices + 3) / 4);
    for (int64_t tile = tl.t; tile < tl.end; tile += tl.step) {
        const int64_t slice = tile * 4 + wv;
        if (slice >= nslices) continue;
        const int64_t row = slice * 64 + lane;
        double v[R];
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = 0.0;
        if (row < nrows) {
            const int s = nsys > 1 ? row_system(row, nsys, sys_ptr) : 0;
            double pp[R], qq[R], xx[R], rr[R];
            vload_nt<double, R>(p + row * R, pp);
            vload_nt<double, R>(q + row * R, qq);
            vload_nt<double, R>(x + row * R, xx);
            vload_nt<double, R>(r + row * R, rr);
            T o[R];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const double d = pq[s * 2 * R + k];
                double alpha = d > 0.0 ? pq[s * 2 * R + R + k] / d : 0.0;
                if (!isfinite(alpha)) alpha = 0.0;
                xx[k] += alpha * pp[k];
                rr[k] -= alpha * qq[k];
                o[k] = (T)rr[k];
                v[k] = rr[k] * rr[k];
            }
            vstore<double, R>(x + row * R, xx);
            vstore<double, R>(r + row * R, rr);
            vstore<T, R>(rt + row * R, o);
        }
        if constexpr (SYS) {
            slice_partials<R>(v, lane, slice, het, spart, rn2);
        } else {
#pragma unroll
            for (int k = 0; k < R; ++k) acc[k] += v[k];
        }
    }
    if constexpr (!SYS) wg_partials<R>(acc, red, partial);
}

// Single-system forms of the vector steps: the [n][R] vectors are streamed as
// flat arrays, two doubles per thread per step (a thread always meets the same
// two right-hand sides, since the grid stride is a multiple of R), which keeps
// registers low and many loads in flight.  Partial sums per workgroup [G][R].
template <int R>
__device__ __forceinline__ void flat_partials(const double (&v)[2], double *red, double *partial) {
    constexpr int K2 = R > 1 ? R / 2 : 1;   // distinct pair positions
    red[threadIdx.x * 2] = v[0];
    red[threadIdx.x * 2 + 1] = v[1];
    __syncthreads();
    for (int h = WG / 2; h >= K2; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[threadIdx.x * 2] += red[(threadIdx.x + h) * 2];
            red[threadIdx.x * 2 + 1] += red[(threadIdx.x + h) * 2 + 1];
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < K2) {
        if constexpr (R == 1) {
            partial[blockIdx.x] = red[0] + red[1];
        } else {
            partial[(int64_t)blockIdx.x * R + 2 * threadIdx.x] = red[threadIdx.x * 2];
            partial[(int64_t)blockIdx.x * R + 2 * threadIdx.x + 1] = red[threadIdx.x * 2 + 1];
        }
    }
}

// Pair range of this workgroup.  One system: a grid-stride over all pairs.
// A batch (sys_wg != null): workgroup b belongs to the system s with
// sys_wg[s] <= b < sys_wg[s+1] and covers a chunk of that system's pairs only,
// so its partial sums and scalars are those of one system.
constexpr int64_t SYS_CHUNK = 4 * WG;   // pairs per workgroup in a batch

struct PairRange {
    int64_t begin, end, stride;
    int sys;
};

template <int R>
__device__ __forceinline__ PairRange pair_range(int64_t npairs, int nsys, const int32_t *__restrict__ sys_wg,
                                                const int64_t *__restrict__ sys_ptr) {
    if (!sys_wg) return {blockIdx.x * (int64_t)WG + threadIdx.x, npairs, (int64_t)gridDim.x * WG, 0};
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sys_wg[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const int64_t p0 = sys_ptr[lo] * R / 2, p1 = sys_ptr[lo + 1] * R / 2;
    const int64_t b = blockIdx.x - sys_wg[lo];
    const int64_t e = p0 + (b + 1) * SYS_CHUNK;
    return {p0 + b * SYS_CHUNK + threadIdx.x, e < p1 ? e : p1, (int64_t)WG, lo};
}

// (z, q) per right-hand side
template <typename T, int R>
__global__ __launch_bounds__(WG) void k_cg_zq_flat(int64_t npairs, int nsys, const int32_t *__restrict__ sys_wg,
                                                   const int64_t *__restrict__ sys_ptr, const T *__restrict__ z,
                                                   const double *__restrict__ q, double *__restrict__ partial) {
    __shared__ double red[2 * WG];
    double v[2] = {0.0, 0.0};
    const PairRange pr = pair_range<R>(npairs, nsys, sys_wg, sys_ptr);
    for (int64_t e2 = pr.begin; e2 < pr.end; e2 += pr.stride) {
        T zz[2];
        double qq[2];
        vload_nt<T, 2>(z + 2 * e2, zz);
        vload_nt<double, 2>(q + 2 * e2, qq);
        v[0] += (double)zz[0] * qq[0];
        v[1] += (double)zz[1] * qq[1];
    }
    flat_partials<R>(v, red, partial);
}

// p = z + beta p (first: p = z), beta = -(z, q_prev) / (p_prev, q_prev)
template <typename T, int R>
__global__ __launch_bounds__(WG) void k_cg_p_flat(int64_t npairs, int nsys, const int32_t *__restrict__ sys_wg,
                                                  const int64_t *__restrict__ sys_ptr, const T *__restrict__ z,
                                                  const double *__restrict__ zq, const double *__restrict__ pq_prev,
                                                  double *__restrict__ p, int first) {
    const PairRange pr = pair_range<R>(npairs, nsys, sys_wg, sys_ptr);
    double beta[2] = {0.0, 0.0};
    if (!first) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int k = (int)((2 * pr.begin + u) % R);
            const double d = pq_prev[pr.sys * 2 * R + k];
            beta[u] = d > 0.0 ? -zq[pr.sys * R + k] / d : 0.0;
            if (!isfinite(beta[u])) beta[u] = 0.0;
        }
    }
    for (int64_t e2 = pr.begin; e2 < pr.end; e2 += pr.stride) {
        T zz[2];
        vload_nt<T, 2>(z + 2 * e2, zz);
        double pp[2] = {0.0, 0.0};
        if (!first) vload_nt<double, 2>(p + 2 * e2, pp);
        pp[0] = (double)zz[0] + beta[0] * pp[0];
        pp[1] = (double)zz[1] + beta[1] * pp[1];
        vstore<double, 2>(p + 2 * e2, pp);
    }
}

// x += alpha p, r -= alpha q, rt = r (working precision), partial r^2
template <typename T, int R>
__global__ __launch_bounds__(WG) void k_cg_update_flat(int64_t npairs, int nsys, const int32_t *__restrict__ sys_wg,
                                                       const int64_t *__restrict__ sys_ptr,
                                                       const double *__restrict__ pq, const double *__restrict__ p,
                                                       const double *__restrict__ q, double *__restrict__ x,
                                                       double *__restrict__ r, T *__restrict__ rt,
                                                       double *__restrict__ partial) {
    __shared__ double red[2 * WG];
    const PairRange pr = pair_range<R>(npairs, nsys, sys_wg, sys_ptr);
    double alpha[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int k = (int)((2 * pr.begin + u) % R);
        const double d = pq[pr.sys * 2 * R + k];
        alpha[u] = d > 0.0 ? pq[pr.sys * 2 * R + R + k] / d : 0.0;
        if (!isfinite(alpha[u])) alpha[u] = 0.0;
    }
    double v[2] = {0.0, 0.0};
    for (int64_t e2 = pr.begin; e2 < pr.end; e2 += pr.stride) {
        double pp[2], qq[2], xx[2], rr[2];
        vload_nt<double, 2>(p + 2 * e2, pp);
        vload_nt<double, 2>(q + 2 * e2, qq);
        vload_nt<double, 2>(x + 2 * e2, xx);
        vload_nt<double, 2>(r + 2 * e2, rr);
        T o[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            xx[u] += alpha[u] * pp[u];
            rr[u] -= alpha[u] * qq[u];
            o[u] = (T)rr[u];
            v[u] += rr[u] * rr[u];
        }
        vstore<double, 2>(x + 2 * e2, xx);
        vstore<double, 2>(r + 2 * e2, rr);
        vstore<T, 2>(rt + 2 * e2, o);
    }
    flat_partials<R>(v, red, partial);
}

// ---------------------------------------------------------------------------
// GMRES vector kernels.  The Krylov basis is kept unnormalised: basis vector i
// is sc[i][col] * vt_i with vt_i stored ([n][R] FP64, leading dimension ld)
// and sc the reciprocal norms, col = system * R + right-hand side.  Vectors
// stream one element per thread and step; a thread always meets the same
// right-hand side (R divides the stride), and in a batch a workgroup covers a
// chunk of one system only, so each thread has one column.
// ---------------------------------------------------------------------------
constexpr int GM_MAXV = 32;             // basis vectors per kernel (restart + 1)
constexpr int64_t GM_CHUNK = 4 * WG;    // elements per workgroup in a batch

// register-array size of the GMRES vector kernels for nv basis vectors
template <class F>
void dispatch_mv(int nv, F &&f) {
    if (nv <= 4) f(std::integral_constant<int, 4>{});
    else if (nv <= 8) f(std::integral_constant<int, 8>{});
    else if (nv <= 16) f(std::integral_constant<int, 16>{});
    else f(std::integral_constant<int, GM_MAXV>{});
}

struct ElemRange {
    int64_t begin, end, stride;
    int sys;
};

template <int R>
__device__ __forceinline__ ElemRange elem_range(int64_t nel, int nsys, const int32_t *__restrict__ sys_wg,
                                                const int64_t *__restrict__ sys_ptr) {
    if (!sys_wg) return {blockIdx.x * (int64_t)WG + threadIdx.x, nel, (int64_t)gridDim.x * WG, 0};
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sys_wg[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const int64_t e0 = sys_ptr[lo] * R, e1 = sys_ptr[lo + 1] * R;
    const int64_t a = e0 + (int64_t)(blockIdx.x - sys_wg[lo]) * GM_CHUNK;
    return {a + threadIdx.x, a + GM_CHUNK < e1 ? a + GM_CHUNK : e1, (int64_t)WG, lo};
}

// Workgroup partial sums of NV values per thread, reduced over the threads of
// one right-hand side (t mod R): partial[blockIdx][i][R].
template <int R, int MV>
__device__ __forceinline__ void gm_partials(const double (&acc)[MV], int nv, double *red,
                                            double *__restrict__ partial) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < MV; ++i) {
        if (i < nv) {   // uniform
            double v = acc[i];
#pragma unroll
            for (int off = 32; off >= R; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane < R) red[(wv * MV + i) * R + lane] = v;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nv * R; e += WG) {
        const int i = e / R, k = e % R;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WG / 64; ++w) s += red[(w * MV + i) * R + k];
        partial[(int64_t)blockIdx.x * nv * R + e] = s;
    }
}

// h_i = (v_i, w) for i < nv
template <typename W, int R, int MV>
__global__ __launch_bounds__(WG) void k_gm_dots(int64_t nel, int nsys, const int32_t *__restrict__ sys_wg,
                                                const int64_t *__restrict__ sys_ptr, int nv,
                                                const double *__restrict__ vt, int64_t ld,
                                                const double *__restrict__ sc, const W *__restrict__ w,
                                                double *__restrict__ partial) {
    __shared__ double red[(WG / 64) * MV * R];
    const ElemRange er = elem_range<R>(nel, nsys, sys_wg, sys_ptr);
    const int col = er.sys * R + (int)(threadIdx.x % R);
    double acc[MV];
#pragma unroll
    for (int i = 0; i < MV; ++i) acc[i] = 0.0;
    for (int64_t e = er.begin; e < er.end; e += er.stride) {
        const double we = (double)w[e];
#pragma unroll
        for (int i = 0; i < MV; ++i)
            if (i < nv) acc[i] += __builtin_nontemporal_load(vt + i * ld + e) * we;
    }
#pragma unroll
    for (int i = 0; i < MV; ++i)
        if (i < nv) acc[i] *= sc[(int64_t)i * nsys * R + col];
    gm_partials<R, MV>(acc, nv, red, partial);
}

// w' = w - sum_i h_i v_i (h[sys][i][R] from the reduction), stored in FP64;
// with DOTS the partial sums of (v_i, w') for i < nv, else of (w', w').
// nv = 0 copies w (converted) and sums its squares.
template <typename W, int R, bool DOTS, int MV>
__global__ __launch_bounds__(WG) void k_gm_update(int64_t nel, int nsys, const int32_t *__restrict__ sys_wg,
                                                  const int64_t *__restrict__ sys_ptr, int nv,
                                                  const double *__restrict__ vt, int64_t ld,
                                                  const double *__restrict__ sc, const double *__restrict__ h,
                                                  const W *__restrict__ w, double *__restrict__ wout,
                                                  double *__restrict__ partial) {
    __shared__ double red[(WG / 64) * MV * R];
    const ElemRange er = elem_range<R>(nel, nsys, sys_wg, sys_ptr);
    const int k = (int)(threadIdx.x % R), col = er.sys * R + k;
    double coef[MV], acc[MV];
#pragma unroll
    for (int i = 0; i < MV; ++i) {
        acc[i] = 0.0;
        coef[i] = i < nv ? h[((int64_t)er.sys * nv + i) * R + k] * sc[(int64_t)i * nsys * R + col] : 0.0;
    }
    for (int64_t e = er.begin; e < er.end; e += er.stride) {
        double v[MV];
        double we = (double)w[e];
#pragma unroll
        for (int i = 0; i < MV; ++i)
            if (i < nv) {
                v[i] = __builtin_nontemporal_load(vt + i * ld + e);
                we -= coef[i] * v[i];
            }
        wout[e] = we;
        if constexpr (DOTS) {
#pragma unroll
            for (int i = 0; i < MV; ++i)
                if (i < nv) acc[i] += v[i] * we;
        } else {
            acc[0] += we * we;
        }
    }
    if constexpr (DOTS) {
#pragma unroll
        for (int i = 0; i < MV; ++i)
            if (i < nv) acc[i] *= sc[(int64_t)i * nsys * R + col];
    }
    gm_partials<R, MV>(acc, DOTS ? nv : 1, red, partial);
}

// x += sum_{i < nv} y[col][i] * basis_i, basis_i = sc_i vt_i (sc != null) or
// the stored preconditioned vectors (sc == null); y is [ncol][ystride]
template <typename B, int R, int MV>
__global__ __launch_bounds__(WG) void k_gm_xupdate(int64_t nel, int nsys, const int32_t *__restrict__ sys_wg,
                                                   const int64_t *__restrict__ sys_ptr, int nv,
                                                   const B *__restrict__ basis, int64_t ld,
                                                   const double *__restrict__ sc, const double *__restrict__ y,
                                                   int ystride, double *__restrict__ x) {
    const ElemRange er = elem_range<R>(nel, nsys, sys_wg, sys_ptr);
    const int col = er.sys * R + (int)(threadIdx.x % R);
    double coef[MV];
#pragma unroll
    for (int i = 0; i < MV; ++i)
        coef[i] = i < nv ? y[(int64_t)col * ystride + i] * (sc ? sc[(int64_t)i * nsys * R + col] : 1.0) : 0.0;
    for (int64_t e = er.begin; e < er.end; e += er.stride) {
        double xe = x[e];
#pragma unroll
        for (int i = 0; i < MV; ++i)
            if (i < nv) xe += coef[i] * (double)__builtin_nontemporal_load(basis + i * ld + e);
        x[e] = xe;
    }
}

// Per-system sums of GMRES partials: out[s][c] = sum over the workgroups of
// system s of partial[b][c], c < W.  Workgroup (s, c-block of 64): wavefront
// w of 16 sums every 16th workgroup with four independent accumulators (loads
// in flight), then the wavefronts are added in order.  Fixed order throughout.
__global__ __launch_bounds__(1024) void k_gm_reduce(int W, int64_t G, const int32_t *__restrict__ sys_wg,
                                                    const double *__restrict__ partial, double *__restrict__ out) {
    __shared__ double red[16][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int s = blockIdx.y;
    const int c = blockIdx.x * 64 + lane;
    const int64_t b0 = sys_wg ? sys_wg[s] : 0, b1 = sys_wg ? sys_wg[s + 1] : G;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    if (c < W) {
        int64_t b = b0 + wv;
        for (; b + 48 < b1; b += 64) {
            v0 += partial[b * W + c];
            v1 += partial[(b + 16) * W + c];
            v2 += partial[(b + 32) * W + c];
            v3 += partial[(b + 48) * W + c];
        }
        for (; b < b1; b += 16) v0 += partial[b * W + c];
    }
    red[wv][lane] = (v0 + v1) + (v2 + v3);
    __syncthreads();
    if (wv == 0 && c < W) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < 16; ++w) t += red[w][lane];
        out[(int64_t)s * W + c] = t;
    }
}

// sc[col] = 1 / sqrt(n2[col]) (0 for a zero or non-finite norm)
__global__ void k_gm_rscale(int ncol, const double *__restrict__ n2, double *__restrict__ sc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    const double v = n2[c];
    sc[c] = (v > 0.0 && isfinite(v)) ? 1.0 / sqrt(v) : 0.0;
}

// out = sc * (A vt) (left GMRES: the V-cycle input, in the working precision)
// or out = b - A x (sc == null, b != null) or A x (both null), FP64 A.
template <typename TO, int R, int NB = 1>
__global__ __launch_bounds__(WG) void k_gm_spmv(int64_t nrows, int64_t nslices, const int64_t *__restrict__ sptr,
                                                const int32_t *__restrict__ slen, const int32_t *__restrict__ scol,
                                                const double *__restrict__ sval, const double *__restrict__ x,
                                                const double *__restrict__ b, const double *__restrict__ sc, int nsys,
                                                const int64_t *__restrict__ sys_ptr, TO *__restrict__ out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const Tiles tl = my_tiles((nslices + 3) / 4);
    for (int64_t tile = tl.t; tile < tl.end; tile += tl.step) {
        const int64_t slice = tile * 4 + wv;
        if (slice >= nslices) continue;
        const int64_t row = slice * 64 + lane;
        if (row >= nrows) continue;
        double ax[R], xo[R];
#pragma unroll
        for (int k = 0; k < R; ++k) ax[k] = 0.0;
        if constexpr (NB > 1) vload<double, R>(x + row * R, xo);
        spmv_row_nb<double, R, false, NB>(scol, sval, sptr[slice] + lane, slen[slice], x, nullptr, 1, row, lane, xo,
                                          ax);
        if (sc) {
            const int s = nsys > 1 ? row_system(row, nsys, sys_ptr) : 0;
#pragma unroll
            for (int k = 0; k < R; ++k) ax[k] *= sc[s * R + k];
        } else if (b) {
            double bb[R];
            vload_nt<double, R>(b + row * R, bb);
#pragma unroll
            for (int k = 0; k < R; ++k) ax[k] = bb[k] - ax[k];
        }
        TO o[R];
#pragma unroll
        for (int k = 0; k < R; ++k) o[k] = (TO)ax[k];
        vstore<TO, R>(out + row * R, o);
    }
}

// out = T(sc * vt) (flexible GMRES: the V-cycle input)
template <typename T, int R>
__global__ __launch_bounds__(WG) void k_gm_scale_cast(int64_t nel, int nsys, const int32_t *__restrict__ sys_wg,
                                                      const int64_t *__restrict__ sys_ptr,
                                                      const double *__restrict__ vt, const double *__restrict__ sc,
                                                      T *__restrict__ out) {
    const ElemRange er = elem_range<R>(nel, nsys, sys_wg, sys_ptr);
    const double f = sc[er.sys * R + (int)(threadIdx.x % R)];
    for (int64_t e = er.begin; e < er.end; e += er.stride) out[e] = (T)(f * vt[e]);
}

// Per-system sums of per-workgroup partials: out[s][k] = sum over the
// workgroups b of system s (sys_wg[s] <= b < sys_wg[s+1]) of partial[b][k].
__global__ __launch_bounds__(256) void k_wg_to_sys(int W, const int32_t *__restrict__ sys_wg,
                                                   const double *__restrict__ partial, double *__restrict__ out) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int64_t e0 = (int64_t)sys_wg[blockIdx.x] * W, e1 = (int64_t)sys_wg[blockIdx.x + 1] * W;
    double s = 0.0;
    for (int64_t e = e0 + t; e < e1; e += 256) s += partial[e];   // W divides 256: component t % W
    red[t] = s;
    __syncthreads();
    for (int h = 128; h >= W; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t < W) out[(int64_t)blockIdx.x * W + t] = red[t];
}

// Fixed-order sum of the partials: out[k] = sum_g partial[g][k]
// One coalesced pass: thread t always accumulates component t % R (R divides
// 1024), then a tree over threads of equal t % R.
__global__ __launch_bounds__(1024) void k_reduce_partials(int64_t G, int R, const double *__restrict__ partial,
                                                          double *__restrict__ out) {
    __shared__ double red[1024];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int64_t e = t; e < G * R; e += 1024) s += partial[e];
    red[t] = s;
    __syncthreads();
    for (int h = 512; h >= R; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t < R) out[t] = red[t];
}

// Per-system squared norms from the slice sums of k_ir_residual<SYS>:
// out[s][k] = sum over the whole slices of system s (spart) + sum over its rows
// in straddling slices (rn2).  One workgroup per system, fixed order.  System
// s owns rows [r0, r1); its whole slices are [fs, fe), the rest of its rows sit
// in straddling slices.
__global__ __launch_bounds__(256) void k_sys_norms(int R, int64_t n, const int64_t *__restrict__ sys_ptr,
                                                   const int32_t *__restrict__ het,
                                                   const double *__restrict__ spart,
                                                   const double *__restrict__ rn2, double *__restrict__ out) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int64_t r0 = sys_ptr[blockIdx.x], r1 = sys_ptr[blockIdx.x + 1];
    const int64_t fs = (r0 + 63) / 64;
    const int64_t fe = (r1 % 64 == 0 || r1 == n) ? (r1 + 63) / 64 : r1 / 64;
    double s = 0.0;
    // R divides 256 and every range starts at a multiple of R: thread t always
    // sums component t % R
    if (fs < fe) {
        for (int64_t e = fs * R + t; e < fe * R; e += 256) s += spart[e];
    }
    auto rows = [&](int64_t a, int64_t b) {
        for (int64_t e = a * R + t; e < b * R; e += 256) {
            const int64_t r = e / R;
            s += rn2[((int64_t)het[r / 64] * 64 + r % 64) * R + e % R];
        }
    };
    if (fs < fe) {
        rows(r0, fs * 64);
        rows(fe * 64 < r1 ? fe * 64 : r1, r1);
    } else {
        rows(r0, r1);
    }
    red[t] = s;
    __syncthreads();
    for (int h = 128; h >= R; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t < R) out[(int64_t)blockIdx.x * R + t] = red[t];
}

template <typename T>
__global__ void k_add_to64(int64_t n, const T *__restrict__ d, double *__restrict__ x) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) x[e] += (double)d[e];
}

template <typename A, typename B>
__global__ void k_convert(int64_t n, const A *__restrict__ a, B *__restrict__ b) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) b[e] = (B)a[e];
}

template <typename T>
__global__ void k_zero(int64_t n, T *__restrict__ a) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) a[e] = T(0);
}

inline unsigned grid_for(int64_t n, int wg = WG) { return (unsigned)ceil_div(n, wg); }

// Workgroups for a tiled (256-row) kernel: one per tile up to the resident
// limit c.sweep_grid (a multiple of 8), beyond which workgroups loop over tiles.
inline unsigned tile_grid(const Ctx &c, int64_t nslices) {
    const int64_t ntiles = ceil_div(nslices, 4);
    return (unsigned)(ntiles <= c.sweep_grid ? ntiles : c.sweep_grid);
}

template <class F>
void dispatch_nb(int nb, F &&f) {
    switch (nb) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 8: f(std::integral_constant<int, 8>{}); break;
        case 16: f(std::integral_constant<int, 16>{}); break;
        default: fail(CS_EINVAL, "block size must be 1, 2, 4, 8 or 16");
    }
}

template <class F>
void dispatch_r(int r, F &&f) {
    switch (r) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 8: f(std::integral_constant<int, 8>{}); break;
        default: fail(CS_EINVAL, "nrhs must be 1, 2, 4 or 8");
    }
}

template <typename T>
const T *sell_val(const Sell &S);
template <>
const double *sell_val<double>(const Sell &S) { return S.val64.get(); }
template <>
const float *sell_val<float>(const Sell &S) { return S.val32.get(); }

template <typename T>
const T *lam_ptr(const Level &L, bool transposed);
template <>
const double *lam_ptr<double>(const Level &L, bool tr) { return tr ? L.lam64T.get() : L.lam64.get(); }
template <>
const float *lam_ptr<float>(const Level &L, bool tr) { return tr ? L.lam32T.get() : L.lam32.get(); }

template <typename T>
const T *pval(const Level &L, bool transposed);
template <>
const double *pval<double>(const Level &L, bool tr) { return tr ? L.pt_val64.get() : L.p_val64.get(); }
template <>
const float *pval<float>(const Level &L, bool tr) { return tr ? L.pt_val32.get() : L.p_val32.get(); }

// Algorithmic bytes of one sweep launch: A's entries with their column index
// (none from a zero guess), the Lambda rows, b and x_out, x_in (all rows of x
// for a colour), and x_c when the interpolation is fused in.
template <typename T, int R>
double sweep_bytes(const Level &L, const Sell &S, bool rowmap, bool zero, bool prol) {
    const int64_t nrows = rowmap ? S.nrows : L.n_active;
    const int64_t nnz = rowmap ? S.nnz : L.act_nnz;
    const double es = sizeof(T);
    return (zero ? 0.0 : nnz * (es + 4.0)) + (double)nrows * L.nb * es + (double)nrows * R * es * 2.0 +
           (zero ? 0.0 : (rowmap ? L.n : nrows) * R * es) + (prol ? (double)L.nc * R * es : 0.0);
}

// acc (natural order, not from zero, no interpolation): the result is added
// into that FP64 vector instead of written to xout (sweep_store).
template <typename T, int R>
void launch_sweep(Ctx &c, const Level &L, const Sell &S, bool rowmap, bool zero, const T *lam, const T *b,
                  const T *xin, T *xout, const T *xc = nullptr, int agg_k = 0, double *acc = nullptr) {
    if (acc && (rowmap || zero || xc)) fail(CS_EINVAL, "accumulating sweep: natural order, not from zero");
    // the natural-order layout is swept over the active rows only (rows of
    // direct segments are solved exactly after the sweeps)
    const int64_t nrows = rowmap ? S.nrows : L.n_active;
    const int64_t nslices = rowmap ? S.nslices : L.act_slices;
    const int64_t nnz = rowmap ? S.nnz : L.act_nnz;
    // levels below SMALL_SLICES slices run one 64-row slice per workgroup,
    // unless the autotuner picked a schedule for the level
    const bool small = L.tune_wgs ? L.tune_wgs == 64 : nslices < SMALL_SLICES;
    unsigned G = small ? (unsigned)std::min<int64_t>(nslices, c.sweep_grid) : tile_grid(c, nslices);
    if (L.tune_grid > 0 && (int64_t)G > L.tune_grid) G = (unsigned)L.tune_grid;
    if (G == 0) return;
    const bool prol = xc != nullptr;
    // trace classes by level size (not by the launch shape the autotuner picks)
    const bool large = nslices >= SMALL_SLICES;
    const int cls = acc ? CS_TRACE_REFINE   // it carries the refinement's update
                        : zero ? CS_TRACE_SWEEP_ZERO
                               : (xc ? CS_TRACE_SWEEP_PROLONG : (large ? CS_TRACE_SWEEP : CS_TRACE_SWEEP_SMALL));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // set for a sampled launch: it times itself
    // an accumulating sweep writes no x_out but reads and writes the FP64 rows
    const double acc_bytes = acc ? (double)nrows * R * (16.0 - sizeof(T)) : 0.0;
    const int slot = trace_begin_launch(c, cls, sweep_bytes<T, R>(L, S, rowmap, zero, prol) + acc_bytes, &ev0, &ev1);
    dispatch_nb(L.nb, [&](auto nbc) {
        constexpr int NB = decltype(nbc)::value;
#define CS_SWEEP_ACC(Z, M, P, ROWS, A)                                                                                 \
    do {                                                                                                               \
        if (small)                                                                                                     \
            hipExtLaunchKernelGGL((k_sweep<T, NB, R, Z, M, P, 64, A>), dim3(G), dim3(64), 0, c.stream, ev0, ev1, 0,   \
                                  nrows, nslices, ROWS, S.slice_ptr.get(), S.slice_len.get(), S.col.get(),            \
                                  sell_val<T>(S), lam, b, xin, xout, xc, agg_k, acc);                                 \
        else                                                                                                           \
            hipExtLaunchKernelGGL((k_sweep<T, NB, R, Z, M, P, WG, A>), dim3(G), dim3(WG), 0, c.stream, ev0, ev1, 0,   \
                                  nrows, nslices, ROWS, S.slice_ptr.get(), S.slice_len.get(), S.col.get(),            \
                                  sell_val<T>(S), lam, b, xin, xout, xc, agg_k, acc);                                 \
    } while (0)
#define CS_SWEEP(Z, M, P, ROWS) CS_SWEEP_ACC(Z, M, P, ROWS, false)
        if (acc) {
            if constexpr (std::is_same<T, double>::value) CS_SWEEP_ACC(false, false, false, nullptr, true);
            else fail(CS_EINVAL, "accumulating sweep: FP64 working precision only");
        } else if (rowmap) {
            if (zero) CS_SWEEP(true, true, false, S.rows.get());
            else CS_SWEEP(false, true, false, S.rows.get());
        } else if (zero) {
            CS_SWEEP(true, false, false, nullptr);
        } else if (prol) {
            CS_SWEEP(false, false, true, nullptr);
        } else {
            CS_SWEEP(false, false, false, nullptr);
        }
#undef CS_SWEEP
#undef CS_SWEEP_ACC
    });
    CS_LAUNCH_CHECK();
}

// Overlapping blocks (Sec. 3.6.2): y = Lambda_l Theta r over the replicated
// slots, r = A x - b (or -b on a zero guess), one thread per (block, slot).
template <typename T, int R>
__global__ void k_ovl_apply(int64_t nblk, int m, const int32_t *__restrict__ nodes, const T *__restrict__ lam,
                            const T *__restrict__ r, int negate, T *__restrict__ y) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= nblk * m) return;
    const int64_t i = e / m;
    const int row = (int)(e % m);
    T acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = T(0);
    const T *lr = lam + (i * m + row) * m;
    for (int u = 0; u < m; ++u) {
        const int node = nodes[i * m + u];
        if (node < 0) continue;
        T rv[R];
        vload<T, R>(r + (int64_t)node * R, rv);
        const T l = lr[u];
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] += l * rv[k];
    }
    if (negate) {
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = -acc[k];
    }
    vstore<T, R>(y + e * R, acc);
}

// x_out = x_in - (1 / theta) Theta^T y (x_in null: a zero guess)
template <typename T, int R>
__global__ void k_ovl_fuse(int64_t n, const int32_t *__restrict__ iptr, const int32_t *__restrict__ iidx,
                           const double *__restrict__ rtheta, const T *__restrict__ y, const T *xin, T *xout) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    T acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = T(0);
    for (int q = iptr[k]; q < iptr[k + 1]; ++q) {
        T yv[R];
        vload<T, R>(y + (int64_t)iidx[q] * R, yv);
#pragma unroll
        for (int j = 0; j < R; ++j) acc[j] += yv[j];
    }
    T xo[R];
    if (xin) vload<T, R>(xin + k * R, xo);
    else {
#pragma unroll
        for (int j = 0; j < R; ++j) xo[j] = T(0);
    }
    const T f = (T)rtheta[k];
#pragma unroll
    for (int j = 0; j < R; ++j) xo[j] -= f * acc[j];
    vstore<T, R>(xout + k * R, xo);
}

// One application of the cascade of level L: x <- S(x, b).  Returns the buffer
// holding the result (additive sweeps alternate between x and alt).  With xc
// given (additive only), the first sweep reads x - P x_c instead of x.  With
// acc64 (additive, at least two steps, or one that is neither from zero nor
// interpolating) the last sweep adds its result into that FP64 vector instead.
template <typename T, int R>
T *apply_cascade(Ctx &c, const Level &L, bool reverse, bool zero_start, const T *b, T *x, T *alt,
                 const T *xc = nullptr, int s_begin = 0, double *acc64 = nullptr) {
    const int64_t nbl = L.B * L.nb * L.nb;
    const int depth = L.depth;
    if (L.ovl_m) {
        // overlapping blocks: forward only (the setup requires FF); residual,
        // blockwise apply over the replicated slots, fused weighted average
        if (reverse || xc) fail(CS_EINVAL, "overlapping-block cascades apply forward without fused interpolation");
        const int64_t m = L.ovl_m, nblk = L.ovl_nblk, lsz = nblk * m * m;
        T *y = reinterpret_cast<T *>(L.w_ovl);
        T *rr = reinterpret_cast<T *>(L.w_rr);
        T *cur = x, *nxt = alt;
        for (int ell = 0; ell < depth; ++ell) {
            const bool zero = zero_start && ell == 0;
            const double es = sizeof(T);
            const int slot = trace_begin(c, zero ? CS_TRACE_SWEEP_ZERO : CS_TRACE_SWEEP_SMALL,
                                         (zero ? 0.0 : L.nnz * (es + 4.0) + 3.0 * L.n * R * es) + lsz * es +
                                             2.0 * nblk * m * R * es + 2.0 * L.n * R * es);
            if (!zero)
                hipLaunchKernelGGL((k_residual<T, R>), dim3(tile_grid(c, L.sell.nslices)), dim3(WG), 0, c.stream,
                                   L.n, L.sell.nslices, L.sell.slice_ptr.get(), L.sell.slice_len.get(),
                                   L.sell.col.get(), sell_val<T>(L.sell), b, cur, rr);
            hipLaunchKernelGGL((k_ovl_apply<T, R>), dim3(grid_for(nblk * m)), dim3(WG), 0, c.stream, nblk, (int)m,
                               L.ovl_nodes.get(), lam_ptr<T>(L, false) + (int64_t)ell * lsz, zero ? b : rr,
                               zero ? 1 : 0, y);
            hipLaunchKernelGGL((k_ovl_fuse<T, R>), dim3(grid_for(L.n)), dim3(WG), 0, c.stream, L.n,
                               L.ovl_inv_ptr.get(), L.ovl_inv_idx.get(), L.ovl_rtheta.get(), (const T *)y,
                               zero ? (const T *)nullptr : (const T *)cur, nxt);
            CS_LAUNCH_CHECK();
            trace_end(c, slot);
            std::swap(cur, nxt);
        }
        return cur;
    }
    if (c.opt.mode == CS_ADDITIVE) {
        // s_begin = 1: step 0 (from zero, into alt) is already on the stream
        T *cur = x, *nxt = alt;
        if (s_begin == 1) std::swap(cur, nxt);
        // the consecutive A-reading sweeps of a large level are timed as one
        // run (one event pair; a timed single launch pays an end-of-kernel
        // release that the untimed ones do not)
        const int s_run = (s_begin == 0 && (zero_start || xc)) ? 1 : s_begin;
        const int s_end = acc64 ? depth - 1 : depth;   // an accumulating last sweep is timed on its own
        int run = -1;
        for (int s = s_begin; s < depth; ++s) {
            if (s == s_run && s_run < s_end && L.act_slices >= SMALL_SLICES)
                run = trace_begin_run(c, CS_TRACE_SWEEP,
                                      (s_end - s_run) * sweep_bytes<T, R>(L, L.sell, false, false, false),
                                      s_end - s_run);
            if (s == s_end) {
                trace_end_run(c, run);
                run = -1;
            }
            const int ell = reverse ? depth - 1 - s : s;
            const T *lam = lam_ptr<T>(L, reverse) + (int64_t)ell * nbl;
            launch_sweep<T, R>(c, L, L.sell, false, zero_start && s == 0, lam, b, cur, nxt, s == 0 ? xc : nullptr,
                               L.agg_k, s == depth - 1 ? acc64 : nullptr);
            std::swap(cur, nxt);
        }
        trace_end_run(c, run);
        return cur;
    }
    // multiplicative: flattened (l, k) sequence, in place
    if (zero_start) {
        hipLaunchKernelGGL(k_zero<T>, dim3(grid_for(L.n_active * R)), dim3(WG), 0, c.stream, L.n_active * R, x);
        CS_LAUNCH_CHECK();
    }
    const int chi = L.chi;
    const int nsteps = depth * chi;
    bool bf16 = false;
    if constexpr (std::is_same<T, float>::value && R == 1) bf16 = use_bf16(c, L);
    // the A-reading colour sweeps of a large level run back to back: timed
    // as one run (as the additive sweeps)
    const int s_run = zero_start ? 1 : 0;
    bool large = bf16 ? L.n >= (1 << 19) : true;
    double run_bytes = 0.0;
    int run_n = 0;
    for (int s = s_run; s < nsteps; ++s) {
        const int k = (reverse ? nsteps - 1 - s : s) % chi;
        if (bf16) {
            if (L.cblk_ptr[k + 1] == L.cblk_ptr[k]) continue;
            run_bytes += bf16_sweep_bytes(L, k, false);
        } else {
            const Sell &S = L.csell[k];
            if (S.nrows == 0) continue;
            large = large && S.nslices >= SMALL_SLICES;
            run_bytes += sweep_bytes<T, R>(L, S, true, false, false);
        }
        ++run_n;
    }
    int run = -1;
    for (int s = 0; s < nsteps; ++s) {
        if (s == s_run && large) run = trace_begin_run(c, CS_TRACE_SWEEP, run_bytes, run_n);
        const int f = reverse ? nsteps - 1 - s : s;
        const int ell = f / chi, k = f % chi;
        if constexpr (std::is_same<T, float>::value && R == 1) {
            if (bf16) {
                bf16_sweep(c, L, ell, k, reverse, zero_start && s == 0, b, x);
                continue;
            }
        }
        const Sell &S = L.csell[k];
        if (S.nrows == 0) continue;
        const T *lam = lam_ptr<T>(L, reverse) + (int64_t)ell * nbl;
        launch_sweep<T, R>(c, L, S, true, zero_start && s == 0, lam, b, x, x);
    }
    trace_end_run(c, run);
    return x;
}

// x_d = A_dd^{-1} b_d on the rows of the direct segments of level L
template <typename T, int R>
void direct_solve(Ctx &c, const Level &L, const T *b, T *x) {
    const int nseg = (int)L.dseg.size() - 1;
    if (nseg <= 0) return;
    const double es = sizeof(T);
    const int slot = trace_begin(c, CS_TRACE_BOTTOM, (double)L.dinv.n * 8.0 + 2.0 * (L.n - L.n_active) * R * es);
    hipLaunchKernelGGL((k_direct_seg<T, R>), dim3(grid_for(L.n - L.n_active, WG / 64)), dim3(WG), 0, c.stream,
                       L.n_active, L.n, nseg, L.dseg_d.get(), L.dinv_off.get(), L.dinv.get(), b, x);
    CS_LAUNCH_CHECK();
    trace_end(c, slot);
}

}  // namespace

// The levels the tail kernel covers: the first level l (the finest included)
// from which every level has at most c.tail_rows rows, every smoothed one is
// additive (no overlapping blocks) with fused transfers and one common block
// size of 1, 2, 4 or 8, and the cycle pre- and post-smooths (the first
// post-smoothing sweep carries the interpolation); -1 when there is none.
int tail_start(const Ctx &c) {
    const int nl = (int)c.lv.size();
    if (c.tail_rows <= 0 || nl < 2 || c.opt.mode != CS_ADDITIVE || !c.fuse_transfers || c.opt.n_pre < 1 ||
        c.opt.n_post < 1)
        return -1;
    const int64_t nb = c.lv[nl - 2].nb;
    if (nb != 1 && nb != 2 && nb != 4 && nb != 8) return -1;
    int from = -1;
    for (int l = nl - 1; l >= 0; --l) {
        const Level &V = c.lv[l];
        bool ok = V.n <= c.tail_rows && !V.ovl_m;
        if (l + 1 < nl) ok = ok && V.agg_k > 0 && V.depth >= 1 && V.nb == nb && V.n_active > 0;
        if (!ok || nl - l > 32) break;   // the kernel tracks the levels in a 32-bit mask
        from = l;
    }
    return from >= 0 && from < nl - 1 ? from : -1;
}

namespace {

template <typename T>
void tail_table(Ctx &c, int nrhs) {
    const int from = tail_start(c);
    c.tail_from = from;
    if (from < 0) return;
    if (c.tail_gen == c.gen && c.tail_prec == c.precision && c.tail_nrhs == nrhs) return;
    std::vector<TailLevel> tab;
    const double es = sizeof(T), vr = (double)nrhs * es;
    double bytes = 0.0;
    for (size_t l = from; l < c.lv.size(); ++l) {
        const Level &L = c.lv[l];
        bytes += (double)L.dinv.n * 8.0 + 2.0 * (L.n - L.n_active) * vr;
        if (l + 1 < c.lv.size()) {
            const double A = L.act_nnz * (es + 4.0), lamb = (double)L.n_active * L.nb * es;
            const double v = (double)L.n_active * vr, sweeps = (double)(c.opt.n_pre + c.opt.n_post) * L.depth;
            bytes += (lamb + 2.0 * v) + (sweeps - 1.0) * (A + lamb + 3.0 * v);   // the first from zero
            bytes += A + 2.0 * v + 2.0 * (double)L.nc * vr;   // residual + restriction, the interpolation read
        }
        TailLevel t{};
        t.n = L.n;
        t.n_active = L.n_active;
        t.nslices = L.act_slices;
        t.nc = L.nc;
        t.nbl = L.B * L.nb * L.nb;
        t.sptr = L.sell.slice_ptr.get();
        t.slen = L.sell.slice_len.get();
        t.scol = L.sell.col.get();
        t.sval = sell_val<T>(L.sell);
        t.lam = l + 1 < c.lv.size() ? lam_ptr<T>(L, false) : nullptr;
        t.lamT = l + 1 < c.lv.size() ? lam_ptr<T>(L, true) : nullptr;
        t.bb = L.w_bb;
        t.xb = L.w_xb;
        t.xt = L.w_xt;
        t.depth = L.depth;
        t.agg_k = L.agg_k;
        t.r_scale = L.r_scale;
        t.nseg = L.dseg.size() > 1 ? (int)L.dseg.size() - 1 : 0;
        t.dseg = L.dseg_d.get();
        t.dinv_off = L.dinv_off.get();
        t.dinv = L.dinv.get();
        tab.push_back(t);
    }
    c.tail_host = tab;
    c.tail_bytes = bytes;
    c.tail_tab.upload(c.tail_host.data(), c.tail_host.size(), c.stream);
    c.tail_gen = c.gen;
    c.tail_prec = c.precision;
    c.tail_nrhs = nrhs;
}

// V-cycle (Alg. 1) from level l down: x_l = V(b_l) from the zero guess, with
// b_l in bb and the result in xb.  Only the active rows are smoothed and
// transferred; the direct segments of every level are solved exactly.
// The first sweep of the next level-0 V-cycle, issued ahead: an additive
// cascade's first pre-smoothing step starts from zero and reads only the
// right-hand side (L0.bb) and Lambda, so it can run while the host checks
// convergence.  Returns whether it was issued.
template <typename T, int R>
bool issue_first_sweep(Ctx &c) {
    if (c.lv.size() < 2 || c.opt.mode != CS_ADDITIVE || c.opt.n_pre < 1) return false;
    if (c.tail_from == 0) return false;   // the whole V-cycle is one tail launch
    Level &L = c.lv[0];
    if (L.ovl_m || L.depth < 1) return false;
    const bool reverse = c.opt.order == CS_RF;
    const int ell = reverse ? L.depth - 1 : 0;
    const T *lam = lam_ptr<T>(L, reverse) + (int64_t)ell * (L.B * L.nb * L.nb);
    launch_sweep<T, R>(c, L, L.sell, false, true, lam, reinterpret_cast<const T *>(L.w_bb),
                       reinterpret_cast<T *>(L.w_xb), reinterpret_cast<T *>(L.w_xt), nullptr, L.agg_k);
    c.spec_pending = true;
    return true;
}

template <typename T, int R>
void vcycle_level(Ctx &c, int l) {
    if (l == c.tail_from && c.tail_gen == c.gen && c.tail_prec == c.precision && c.tail_nrhs == R) {
        const int nlev = (int)c.lv.size() - l;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        const int slot = trace_begin_launch(c, CS_TRACE_TAIL, c.tail_bytes, &ev0, &ev1);
        (void)slot;
        dispatch_nb((int)c.lv[l].nb, [&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            if constexpr (NB <= 8)
                hipExtLaunchKernelGGL((k_tail_vcycle<T, NB, R>), dim3(1), dim3(tail_wg<T, R>()), 0, c.stream, ev0, ev1, 0,
                                      (const TailLevel *)c.tail_tab.get(), nlev, c.opt.n_pre, c.opt.n_post,
                                      c.opt.order == CS_RF ? 1 : 0);
        });
        CS_LAUNCH_CHECK();
        return;
    }
    Level &L = c.lv[l];
    T *xb = reinterpret_cast<T *>(L.w_xb);
    T *xt = reinterpret_cast<T *>(L.w_xt);
    T *bb = reinterpret_cast<T *>(L.w_bb);
    T *rr = reinterpret_cast<T *>(L.w_rr);
    const double es = sizeof(T);
    if (l + 1 == (int)c.lv.size()) {
        direct_solve<T, R>(c, L, bb, xb);
        return;
    }
    Level &C = c.lv[l + 1];
    const int64_t na = L.n_active;
    T *x = xb, *alt = xt;
    const bool rf = c.opt.order == CS_RF;
    for (int a = 0; a < c.opt.n_pre; ++a) {
        const int s0 = (l == 0 && a == 0 && c.spec_pending) ? 1 : 0;
        if (s0) c.spec_pending = false;
        T *res = apply_cascade<T, R>(c, L, rf, a == 0, bb, x, alt, nullptr, s0);
        if (res != x) std::swap(x, alt);
    }
    // restricted residual
    const bool fused = c.fuse_transfers && L.agg_k > 0;
    int slot = trace_begin(c, CS_TRACE_RESIDUAL,
                           L.act_nnz * (es + 4.0) + (fused ? 2.0 : 3.0) * na * R * es +
                               (fused ? 0.0 : L.p_nnz * (es + 4.0) + na * R * es) + L.nc * R * es);
    if (fused) {
        dispatch_nb((int)L.nb, [&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            hipLaunchKernelGGL((k_residual_restrict<T, R, NB>), dim3(tile_grid(c, L.act_slices)), dim3(WG), 0, c.stream, na,
                               L.act_slices, L.sell.slice_ptr.get(), L.sell.slice_len.get(), L.sell.col.get(),
                               sell_val<T>(L.sell), bb, x, L.agg_k, L.nc, (T)L.r_scale,
                               reinterpret_cast<T *>(C.w_bb));
        });
    } else {
        // the residual that the coarse level sees is formed in the working
        // precision's vector type with the FP32/FP64 copy of A, also when the
        // sweeps run in BF16: BF16 rounding of A here would corrupt the smooth
        // error components that the coarse-grid correction must remove
        hipLaunchKernelGGL((k_residual<T, R>), dim3(tile_grid(c, L.act_slices)), dim3(WG), 0, c.stream, na,
                           L.act_slices, L.sell.slice_ptr.get(), L.sell.slice_len.get(), L.sell.col.get(),
                           sell_val<T>(L.sell), bb, x, rr);
        hipLaunchKernelGGL((k_restrict_sell<T, R>), dim3(tile_grid(c, L.ptsell.nslices)), dim3(WG), 0, c.stream,
                           L.nc, L.ptsell.nslices, L.ptsell.slice_ptr.get(), L.ptsell.slice_len.get(),
                           L.ptsell.col.get(), sell_val<T>(L.ptsell), (T)L.r_scale, rr,
                           reinterpret_cast<T *>(C.w_bb));
    }
    CS_LAUNCH_CHECK();
    trace_end(c, slot);
    vcycle_level<T, R>(c, l + 1);
    const T *xc = reinterpret_cast<const T *>(C.w_xb);
    const bool fuse_prol = fused && c.opt.mode == CS_ADDITIVE && c.opt.n_post > 0;
    if (!fuse_prol) {
        slot = trace_begin(c, CS_TRACE_PROLONG, L.p_nnz * (es + 4.0) + 2.0 * na * R * es + L.nc * R * es);
        hipLaunchKernelGGL((k_prolong_sell<T, R>), dim3(tile_grid(c, ceil_div(na, 64))), dim3(WG), 0, c.stream,
                           na, ceil_div(na, 64), L.psell.slice_ptr.get(), L.psell.slice_len.get(), L.psell.col.get(),
                           sell_val<T>(L.psell), xc, x);
        CS_LAUNCH_CHECK();
        trace_end(c, slot);
    }
    // the outer refinement's x += x_0 folded into the last fine-level sweep
    // (c.acc_x64): only where that sweep is the V-cycle's last write on level
    // 0 - additive, not the interpolating first post-sweep, no direct segments
    double *acc = nullptr;
    if (l == 0 && c.acc_x64 && c.opt.mode == CS_ADDITIVE && !L.ovl_m && L.depth >= 1 && L.dseg.size() <= 1 &&
        c.opt.n_post >= 1 && !(fuse_prol && c.opt.n_post == 1 && L.depth == 1))
        acc = c.acc_x64;
    for (int a = 0; a < c.opt.n_post; ++a) {
        T *res = apply_cascade<T, R>(c, L, false, false, bb, x, alt, (fuse_prol && a == 0) ? xc : nullptr, 0,
                                     a == c.opt.n_post - 1 ? acc : nullptr);
        if (res != x) std::swap(x, alt);
    }
    if (acc) {
        c.acc_done = true;   // x_0 is in c.acc_x64, not in xb
        return;
    }
    if (x != xb) {
        CS_HIP(hipMemcpyAsync(xb, x, na * R * sizeof(T), hipMemcpyDeviceToDevice, c.stream));
    }
    direct_solve<T, R>(c, L, bb, xb);
}

template <class F>
void dispatch_prec(int prec, F &&f) {
    if (prec == CS_FP64) f((double *)nullptr);
    else f((float *)nullptr);
}

}  // namespace

// Point every level's V-cycle workspace at the context's own buffers (after
// a call that ran on the static scratch array).
static void use_own_workspace(Ctx &c) {
    for (Level &L : c.lv) {
        L.w_xb = L.xb.get();
        L.w_xt = L.xt.get();
        L.w_bb = L.bb.get();
        L.w_rr = L.rr.get();
        L.w_ovl = L.ovl_y.get();
    }
    if (c.ws_scratch) c.gen++;   // captured graphs hold the scratch addresses
    c.ws_scratch = false;
}

static void prepare_tail(Ctx &c, int nrhs) {
    if (c.precision == CS_FP64) tail_table<double>(c, nrhs);
    else tail_table<float>(c, nrhs);
}

void ensure_workspace(Ctx &c, int nrhs) {
    const int prec = c.precision;
    if (c.ws_nrhs == nrhs && c.ws_prec == prec) {
        if (c.ws_scratch) use_own_workspace(c);
        prepare_tail(c, nrhs);
        return;
    }
    const size_t es = prec == CS_FP64 ? sizeof(double) : sizeof(float);
    for (Level &L : c.lv) {
        const size_t bytes = (size_t)L.n * nrhs * es;
        L.xb.alloc(bytes);
        L.xt.alloc(bytes);
        L.bb.alloc(bytes);
        L.rr.alloc(bytes);
        if (L.ovl_m) L.ovl_y.alloc((size_t)L.ovl_nblk * L.ovl_m * nrhs * es);
    }
    c.ws_scratch = true;   // forces the pointer update below
    use_own_workspace(c);
    const int64_t G = std::min<int64_t>(ceil_div(c.lv[0].sell.nslices, 4), IR_GRID);
    c.ir_partial.alloc(std::max<int64_t>(G, 1) * 2 * nrhs);   // up to two dot products per RHS
    const int64_t nsys = c.sys_ptr.empty() ? 1 : (int64_t)c.sys_ptr.size() - 1;
    c.ir_norm.alloc(2 * nsys * nrhs);
    if (nsys > 1) {
        c.sys_spart.alloc((size_t)c.lv[0].sell.nslices * 2 * nrhs);
        c.rn2.alloc((size_t)std::max<int64_t>(c.n_het, 1) * 64 * 2 * nrhs);
    } else {
        c.sys_spart.release();
        c.rn2.release();
    }
    if ((size_t)(2 * nsys * nrhs) > c.h_norm_cap) {
        if (c.h_norm) CS_HIP(hipHostFree(c.h_norm));
        c.h_norm = nullptr;
        c.h_norm_cap = 0;
        CS_HIP(hipHostMalloc(reinterpret_cast<void **>(&c.h_norm), 2 * nsys * nrhs * sizeof(double)));
        c.h_norm_cap = 2 * nsys * nrhs;
    }
    c.ws_nrhs = nrhs;
    c.gen++;
    c.ws_prec = prec;
    prepare_tail(c, nrhs);
}

static void vcycle_run(Ctx &c, const double *b, double *x, int nrhs) {
    Level &L0 = c.lv[0];
    const int64_t n = L0.n * nrhs;
    dispatch_prec(c.precision, [&](auto tp) {
        using T = std::remove_pointer_t<decltype(tp)>;
        hipLaunchKernelGGL((k_convert<double, T>), dim3(grid_for(n)), dim3(WG), 0, c.stream, n, b,
                           reinterpret_cast<T *>(L0.w_bb));
        dispatch_r(nrhs, [&](auto rc) { vcycle_level<T, decltype(rc)::value>(c, 0); });
        hipLaunchKernelGGL((k_convert<T, double>), dim3(grid_for(n)), dim3(WG), 0, c.stream, n,
                           reinterpret_cast<const T *>(L0.w_xb), x);
        CS_LAUNCH_CHECK();
    });
}

void vcycle_apply(Ctx &c, const double *b, double *x, int nrhs) {
    ensure_workspace(c, nrhs);
    vcycle_run(c, b, x, nrhs);
}

// Bytes of V-cycle workspace for nrhs right-hand sides in the working
// precision: x, its double buffer, b and r of every level (+ the replicated
// slots of overlapping-block levels), each range 256-byte aligned.
size_t vcycle_workspace_bytes(const Ctx &c, int nrhs) {
    const size_t es = c.precision == CS_FP64 ? sizeof(double) : sizeof(float);
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t tot = 0;
    for (const Level &L : c.lv) {
        tot += 4 * up((size_t)L.n * nrhs * es);
        if (L.ovl_m) tot += up((size_t)L.ovl_nblk * L.ovl_m * nrhs * es);
    }
    return tot;
}

// x = V b with the level workspace carved out of `scratch` (device memory of
// at least vcycle_workspace_bytes): the same kernels as vcycle_apply, no
// allocation, no event tracing, no synchronisation.  The context's own
// buffers are restored by the next ensure_workspace.
void vcycle_apply_scratch(Ctx &c, const double *b, double *x, int nrhs, unsigned char *scratch) {
    const size_t es = c.precision == CS_FP64 ? sizeof(double) : sizeof(float);
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = scratch + off;
        off += up(bytes);
        return p;
    };
    for (Level &L : c.lv) {
        const size_t bytes = (size_t)L.n * nrhs * es;
        L.w_xb = reinterpret_cast<char *>(take(bytes));
        L.w_xt = reinterpret_cast<char *>(take(bytes));
        L.w_bb = reinterpret_cast<char *>(take(bytes));
        L.w_rr = reinterpret_cast<char *>(take(bytes));
        L.w_ovl = L.ovl_m ? take((size_t)L.ovl_nblk * L.ovl_m * nrhs * es) : nullptr;
    }
    c.ws_scratch = true;
    c.gen++;   // no captured graph may keep these addresses
    const bool tr = c.tr.on;
    c.tr.on = false;
    try {
        vcycle_run(c, b, x, nrhs);
    } catch (...) {
        c.tr.on = tr;
        throw;
    }
    c.tr.on = tr;
}

// Sweep launch schedules per level, picked by measurement: one application of
// the level's cascade (its real operator, smoothers and colour layout) is
// timed with HIP events for every candidate schedule, 64 or 256 rows per
// workgroup with a workgroup per tile or a capped, looping grid (caps are
// multiples of 8 so that every XCD sweeps whole tile ranges); the median of
// five applications decides.  ms[l] receives the best time of level l.
void autotune(Ctx &c, int nrhs, double *ms) {
    ensure_workspace(c, nrhs);
    const bool tr = c.tr.on;
    c.tr.on = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CS_HIP(hipEventCreate(&e0));
    CS_HIP(hipEventCreate(&e1));
    struct Cand {
        int wgs;
        int64_t grid;
    };
    try {
        dispatch_prec(c.precision, [&](auto tp) {
            using T = std::remove_pointer_t<decltype(tp)>;
            dispatch_r(nrhs, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                for (size_t l = 0; l < c.lv.size(); ++l) {
                    Level &L = c.lv[l];
                    if (ms) ms[l] = 0.0;
                    if (L.depth <= 0 || L.n_active == 0 || l + 1 == c.lv.size()) continue;
                    const int64_t n = L.n * R;
                    T *b = reinterpret_cast<T *>(L.w_bb), *x = reinterpret_cast<T *>(L.w_xb),
                      *alt = reinterpret_cast<T *>(L.w_xt);
                    hipLaunchKernelGGL(k_zero<T>, dim3(grid_for(n)), dim3(WG), 0, c.stream, n, b);
                    hipLaunchKernelGGL(k_zero<T>, dim3(grid_for(n)), dim3(WG), 0, c.stream, n, x);
                    CS_LAUNCH_CHECK();
                    const int64_t ns = std::max<int64_t>(L.act_slices, 1), nt = ceil_div(ns, 4);
                    std::vector<Cand> cands{{64, 0}, {256, 0}};
                    for (int64_t g : {1024, 2048, 4096})
                        for (int w : {64, 256})
                            if (g < (w == 64 ? ns : nt)) cands.push_back({w, g});
                    double best = 1e30;
                    Cand pick{0, 0};
                    for (const Cand &cd : cands) {
                        L.tune_wgs = cd.wgs;
                        L.tune_grid = cd.grid;
                        (void)apply_cascade<T, R>(c, L, false, false, b, x, alt);   // warm-up
                        std::vector<float> t(5);
                        for (float &v : t) {
                            CS_HIP(hipEventRecord(e0, c.stream));
                            (void)apply_cascade<T, R>(c, L, false, false, b, x, alt);
                            CS_HIP(hipEventRecord(e1, c.stream));
                            CS_HIP(hipEventSynchronize(e1));
                            CS_HIP(hipEventElapsedTime(&v, e0, e1));
                        }
                        std::sort(t.begin(), t.end());
                        if (t[2] < best) {
                            best = t[2];
                            pick = cd;
                        }
                    }
                    L.tune_wgs = pick.wgs;
                    L.tune_grid = pick.grid;
                    if (ms) ms[l] = best;
                }
            });
        });
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        c.tr.on = tr;
        throw;
    }
    CS_HIP(hipEventDestroy(e0));
    CS_HIP(hipEventDestroy(e1));
    c.tr.on = tr;
    c.gen++;   // captured graphs hold the old launch shapes
}

void smooth_apply(Ctx &c, int level, bool reverse, const double *b, double *x, int nrhs) {
    ensure_workspace(c, nrhs);
    Level &L = c.lv[level];
    const int64_t n = L.n * nrhs;
    dispatch_prec(c.precision, [&](auto tp) {
        using T = std::remove_pointer_t<decltype(tp)>;
        T *bb = reinterpret_cast<T *>(L.w_bb);
        T *xb = reinterpret_cast<T *>(L.w_xb);
        T *xt = reinterpret_cast<T *>(L.w_xt);
        hipLaunchKernelGGL((k_convert<double, T>), dim3(grid_for(n)), dim3(WG), 0, c.stream, n, b, bb);
        hipLaunchKernelGGL((k_convert<double, T>), dim3(grid_for(n)), dim3(WG), 0, c.stream, n, (const double *)x, xb);
        T *res = nullptr;
        dispatch_r(nrhs, [&](auto rc) {
            res = apply_cascade<T, decltype(rc)::value>(c, L, reverse, false, bb, xb, xt);
        });
        // rows of direct segments are not smoothed: they keep their input values
        if (res != xb && L.n_active < L.n) {
            const int64_t off = L.n_active * nrhs;
            CS_HIP(hipMemcpyAsync(res + off, xb + off, (n - off) * sizeof(T), hipMemcpyDeviceToDevice, c.stream));
        }
        hipLaunchKernelGGL((k_convert<T, double>), dim3(grid_for(n)), dim3(WG), 0, c.stream, n, (const T *)res, x);
        CS_LAUNCH_CHECK();
    });
}

namespace {

// Convergence bookkeeping shared by the refinement and Krylov drivers: every
// (system, right-hand side) residual is measured against its own ||b||, and
// the iteration stops when the largest relative residual reaches rtol.
struct Monitor {
    Ctx &c;
    int nsys, R;
    double rtol;
    std::vector<double> hist, bn2;
    Monitor(Ctx &cc, int ns, int r, double tol) : c(cc), nsys(ns), R(r), rtol(tol), bn2((size_t)ns * r, 1.0) {
        c.sys_iters.assign(nsys, -1);
        c.sys_rel.assign(nsys, NAN);
    }
    // hn: squared residual norms [nsys][R], followed (at it == 0) by those of b
    double record(int it, const double *hn) {
        if (it == 0)
            for (int e = 0; e < nsys * R; ++e) bn2[e] = hn[nsys * R + e] > 0 ? hn[nsys * R + e] : 1.0;
        double rel = 0.0;
        bool bad = false;
        for (int q = 0; q < nsys; ++q) {
            double rq = 0.0;
            for (int k = 0; k < R; ++k) {
                const double v = std::sqrt(hn[q * R + k] / bn2[q * R + k]);
                if (!std::isfinite(v) || v > 1e6) bad = true;   // diverged
                rq = std::max(rq, v);
            }
            c.sys_rel[q] = rq;
            if (c.sys_iters[q] < 0 && rq <= rtol) c.sys_iters[q] = it;
            rel = std::max(rel, rq);
        }
        hist.push_back(bad ? NAN : rel);
        return hist.back();
    }
    void finish(int it, float ms, cs_info *info, double *history) {
        for (int q = 0; q < nsys; ++q)
            if (c.sys_iters[q] < 0) c.sys_iters[q] = it;
        if (history)
            for (size_t q = 0; q < hist.size(); ++q) history[q] = hist[q];
        if (!info) return;
        info->iterations = it;
        info->rel_res = hist.back();
        info->solve_ms = ms;
        info->setup_ms = c.setup_ms;
        info->singular_blocks = c.singular;
        // least-squares slope of log r_i over i = 1..K (Sec. 3.1)
        const int K = (int)hist.size() - 1;
        double rho = NAN;
        if (K >= 2) {
            double si = 0, sy = 0, sii = 0, siy = 0;
            for (int q = 1; q <= K; ++q) {
                const double y = std::log(hist[q]);
                si += q;
                sy += y;
                sii += (double)q * q;
                siy += q * y;
            }
            rho = std::exp((K * siy - si * sy) / (K * sii - si * si));
        } else if (K == 1) {
            rho = hist[1] / hist[0];
        }
        info->rho = rho;
        // geometric mean rate over the whole history, and eta of the regression rate
        info->rho_geo = K >= 1 ? std::pow(hist[K] / hist[0], 1.0 / K) : NAN;
        // no decade is ever reached at rho >= 1: eta is infinite there
        info->eta = (rho > 0.0 && rho < 1.0) ? std::log(0.1) / std::log(rho) : (rho >= 1.0 ? INFINITY : NAN);
    }
};

}  // namespace

namespace {

// With graph replay the solve runs on the context's own non-blocking stream
// (capture needs one), ordered after the caller's stream on entry and before
// it on exit.  Replay is off while event tracing is on.
struct SolveStream {
    Ctx &c;
    hipStream_t user;
    bool on;
    SolveStream(Ctx &cc, bool enable) : c(cc), user(cc.stream), on(enable) {
        if (!on) return;
        if (!c.work) CS_HIP(hipStreamCreateWithFlags(&c.work, hipStreamNonBlocking));
        CS_HIP(hipEventRecord(c.ev_in, user));
        CS_HIP(hipStreamWaitEvent(c.work, c.ev_in, 0));
        c.stream = c.work;
    }
    ~SolveStream() {
        if (!on) return;
        (void)hipEventRecord(c.ev_out, c.stream);
        (void)hipStreamWaitEvent(user, c.ev_out, 0);
        c.stream = user;
    }
};

// The device work of one outer iteration after the host's convergence check:
// issued eagerly, or replayed as one graph launch (captured on first use and
// whenever the key changes: other vectors, right-hand-side count, precision,
// method, or device buffers).  Replays issue exactly the captured launches,
// so both forms give identical results.
template <class F>
void run_iteration(Ctx &c, bool graphs, const Ctx::GraphKey &key, F &&body) {
    if (!graphs) {
        body();
        return;
    }
    if (!c.gexec || !(key == c.gkey)) {
        graph_release(c);
        CS_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
        try {
            body();
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(c.stream, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        CS_HIP(hipStreamEndCapture(c.stream, &c.graph));
        CS_HIP(hipGraphInstantiate(&c.gexec, c.graph, nullptr, nullptr, 0));
        c.gkey = key;
    }
    CS_HIP(hipGraphLaunch(c.gexec, c.stream));
}

// however a solve loop ends, no later V-cycle skips its first sweep
struct SpecReset {
    Ctx &c;
    ~SpecReset() { c.spec_pending = false; }
};

}  // namespace

// Eager launches or graph replay for the outer iterations, by measurement:
// one V-cycle issued eagerly and the same V-cycle replayed from a captured
// graph are each timed five times on the work stream (median); replay is kept
// when it is faster.  Returns the two medians in ms (eager, graph).
void tune_graphs(Ctx &c, int nrhs, double *eager_ms, double *graph_ms) {
    ensure_workspace(c, nrhs);
    const bool tr = c.tr.on;
    c.tr.on = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    auto cleanup = [&]() {
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        c.tr.on = tr;
    };
    try {
        SolveStream ss(c, true);
        CS_HIP(hipEventCreate(&e0));
        CS_HIP(hipEventCreate(&e1));
        dispatch_prec(c.precision, [&](auto tp) {
            using T = std::remove_pointer_t<decltype(tp)>;
            dispatch_r(nrhs, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                auto median = [&](auto &&issue) {
                    issue();   // warm-up
                    std::vector<float> t(5);
                    for (float &v : t) {
                        CS_HIP(hipEventRecord(e0, c.stream));
                        issue();
                        CS_HIP(hipEventRecord(e1, c.stream));
                        CS_HIP(hipEventSynchronize(e1));
                        CS_HIP(hipEventElapsedTime(&v, e0, e1));
                    }
                    std::sort(t.begin(), t.end());
                    return (double)t[2];
                };
                *eager_ms = median([&]() { vcycle_level<T, R>(c, 0); });
                CS_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
                try {
                    vcycle_level<T, R>(c, 0);
                } catch (...) {
                    hipGraph_t junk = nullptr;
                    (void)hipStreamEndCapture(c.stream, &junk);
                    if (junk) (void)hipGraphDestroy(junk);
                    throw;
                }
                CS_HIP(hipStreamEndCapture(c.stream, &g));
                CS_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
                *graph_ms = median([&]() { CS_HIP(hipGraphLaunch(ge, c.stream)); });
            });
        });
        CS_HIP(hipStreamSynchronize(c.stream));
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
    c.use_graphs = *graph_ms < *eager_ms;
}

// The tail V-cycle's size limit, picked by measurement: one V-cycle is timed
// (median of five) with the tail off and with every limit that starts it at
// another level (the sizes of the levels of at most 65536 rows); the fastest
// is kept.  ms[k] / rows[k] receive the candidates' times and limits.
int tune_tail(Ctx &c, int nrhs, int64_t *rows, double *ms, int cap) {
    std::vector<int64_t> cand{0};
    for (size_t l = 0; l < c.lv.size(); ++l)
        if (c.lv[l].n <= 65536 && std::find(cand.begin(), cand.end(), c.lv[l].n) == cand.end())
            cand.push_back(c.lv[l].n);
    const int64_t keep = c.tail_rows;
    const bool tr = c.tr.on;
    c.tr.on = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        c.tr.on = tr;
    };
    int nout = 0;
    try {
        CS_HIP(hipEventCreate(&e0));
        CS_HIP(hipEventCreate(&e1));
        int64_t best = 0;
        double best_ms = 0.0;
        std::vector<int> seen_from;
        for (int64_t v : cand) {
            c.tail_rows = v;
            c.tail_gen = ~uint64_t(0);
            ensure_workspace(c, nrhs);
            const int from = v ? c.tail_from : -1;
            if (v && (from < 0 || std::find(seen_from.begin(), seen_from.end(), from) != seen_from.end())) continue;
            seen_from.push_back(from);
            double t_ms = 0.0;
            dispatch_prec(c.precision, [&](auto tp) {
                using T = std::remove_pointer_t<decltype(tp)>;
                dispatch_r(nrhs, [&](auto rc) {
                    constexpr int R = decltype(rc)::value;
                    vcycle_level<T, R>(c, 0);   // warm-up
                    std::vector<float> t(5);
                    for (float &u : t) {
                        CS_HIP(hipEventRecord(e0, c.stream));
                        vcycle_level<T, R>(c, 0);
                        CS_HIP(hipEventRecord(e1, c.stream));
                        CS_HIP(hipEventSynchronize(e1));
                        CS_HIP(hipEventElapsedTime(&u, e0, e1));
                    }
                    std::sort(t.begin(), t.end());
                    t_ms = t[2];
                });
            });
            if (nout < cap) {
                if (rows) rows[nout] = v;
                if (ms) ms[nout] = t_ms;
            }
            ++nout;
            if (v == 0 || t_ms < best_ms) {
                best = v;
                best_ms = t_ms;
            }
        }
        c.tail_rows = best;
    } catch (...) {
        c.tail_rows = keep;
        cleanup();
        throw;
    }
    cleanup();
    c.tail_gen = ~uint64_t(0);
    c.gen++;
    return nout;
}

void solve_ir(Ctx &c, const double *b, double *x, int nrhs, double rtol, int maxit, cs_info *info,
              double *history, cs_status *st) {
    ensure_workspace(c, nrhs);
    Level &L0 = c.lv[0];
    const Sell &S = L0.sell;
    const int64_t n = L0.n * nrhs;
    const int64_t G = std::min<int64_t>(ceil_div(S.nslices, 4), IR_GRID);
    const int nsys = c.sys_ptr.empty() ? 1 : (int)c.sys_ptr.size() - 1;
    const double *hn = c.h_norm;
    *st = CS_OK;
    const bool graphs = c.use_graphs && !c.tr.on;
    SolveStream ss(c, graphs);
    CS_HIP(hipEventRecord(c.ev0, c.stream));
    dispatch_prec(c.precision, [&](auto tp) {
        using T = std::remove_pointer_t<decltype(tp)>;
        dispatch_r(nrhs, [&](auto rc) {
            constexpr int R = decltype(rc)::value;
            const double ir_bytes = S.nnz * 12.0 + (double)L0.n * R * (16.0 + sizeof(T));
            const double up_bytes = (double)L0.n * R * (16.0 + sizeof(T));
            // squared norms of r (and of b, at offset nsys*R): per system in a batch
            const bool batch = nsys > 1;
            auto norms = [&](const double *xx, T *rt, double *out) {
                if (batch) {
                    dispatch_nb((int)L0.nb, [&](auto nbc) {
                        constexpr int NB = decltype(nbc)::value;
                        hipLaunchKernelGGL((k_ir_residual<T, R, true, NB>), dim3(G), dim3(WG), 0, c.stream, S.nrows,
                                           S.nslices, S.slice_ptr.get(), S.slice_len.get(), S.col.get(), S.val64.get(), b,
                                           xx, rt, (double *)nullptr, c.sys_het.get(), c.sys_spart.get(), c.rn2.get());
                    });
                    hipLaunchKernelGGL(k_sys_norms, dim3(nsys), dim3(256), 0, c.stream, R, S.nrows,
                                       c.sys_ptr_d.get(), c.sys_het.get(), c.sys_spart.get(), c.rn2.get(), out);
                } else {
                    dispatch_nb((int)L0.nb, [&](auto nbc) {
                        constexpr int NB = decltype(nbc)::value;
                        hipLaunchKernelGGL((k_ir_residual<T, R, false, NB>), dim3(G), dim3(WG), 0, c.stream, S.nrows,
                                           S.nslices, S.slice_ptr.get(), S.slice_len.get(), S.col.get(), S.val64.get(), b,
                                           xx, rt, c.ir_partial.get(), (const int32_t *)nullptr, (double *)nullptr,
                                           (double *)nullptr);
                    });
                    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(1024), 0, c.stream, G, R, c.ir_partial.get(),
                                       out);
                }
                CS_LAUNCH_CHECK();
            };
            auto residual = [&]() {
                const int slot = trace_begin(c, CS_TRACE_REFINE, ir_bytes);
                norms(x, reinterpret_cast<T *>(L0.w_bb), c.ir_norm.get());
                trace_end(c, slot);
            };
            // one refinement iteration after the check: d = V r, x += d, r = b - A x
            auto iteration = [&]() {
                // in FP64 the V-cycle's last fine sweep adds d into x where it can
                // (128^3, 8 RHS: 52.2 -> 49.9 ms); in FP32 the accumulating
                // sweep holds more registers than the plain one (three waves per
                // SIMD instead of four) and the solve gained nothing (24.35 vs
                // 24.39 ms), so FP32 keeps the separate pass
                struct AccScope {
                    Ctx &c;
                    ~AccScope() { c.acc_x64 = nullptr; }   // also when a launch fails
                } scope{c};
                c.acc_x64 = std::is_same<T, double>::value ? x : nullptr;
                c.acc_done = false;
                vcycle_level<T, R>(c, 0);
                c.acc_x64 = nullptr;
                if (!c.acc_done) {
                    const int slot = trace_begin(c, CS_TRACE_REFINE, up_bytes);
                    hipLaunchKernelGGL((k_add_to64<T>), dim3(grid_for(n)), dim3(WG), 0, c.stream, n,
                                       reinterpret_cast<const T *>(L0.w_xb), x);
                    CS_LAUNCH_CHECK();
                    trace_end(c, slot);
                }
                residual();
            };
            // ||b||^2, x = 0, first residual
            norms(nullptr, (T *)nullptr, c.ir_norm.get() + nsys * R);
            hipLaunchKernelGGL(k_zero<double>, dim3(grid_for(n)), dim3(WG), 0, c.stream, n, x);
            CS_LAUNCH_CHECK();
            residual();
            Monitor mon(c, nsys, R, rtol);
            int it = 0;
            if (!c.ev_norm) CS_HIP(hipEventCreateWithFlags(&c.ev_norm, hipEventDisableTiming));
            SpecReset spec_reset{c};
            const Ctx::GraphKey key{b, x, R, c.precision, 0, c.gen, 0};
            for (;; ++it) {
                CS_HIP(hipMemcpyAsync(c.h_norm, c.ir_norm.get(), 2 * nsys * R * sizeof(double),
                                      hipMemcpyDeviceToHost, c.stream));
                CS_HIP(hipEventRecord(c.ev_norm, c.stream));
                // the next V-cycle's first sweep reads only r and Lambda: issued
                // while the host waits for the norms (one wasted sweep when this
                // check ends the solve)
                if (it < maxit) issue_first_sweep<T, R>(c);
                CS_HIP(hipEventSynchronize(c.ev_norm));
                const double rel = mon.record(it, hn);
                if (std::isnan(rel)) {
                    *st = CS_ENAN;
                    break;
                }
                if (rel <= rtol) break;
                if (it == maxit) {
                    *st = CS_ENOCONV;
                    break;
                }
                run_iteration(c, graphs, key, iteration);
                c.spec_pending = false;
            }
            trace_flush(c);
            CS_HIP(hipEventRecord(c.ev1, c.stream));
            CS_HIP(hipEventSynchronize(c.ev1));
            float ms = 0;
            CS_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
            mon.finish(it, ms, info, history);
        });
    });
}

// Flexible conjugate gradients preconditioned by one V-cycle (FCG(1): the new
// direction is z minus its A-projection on the previous one), FP64 vectors
// and scalars, the V-cycle in the working precision.  Per (system, RHS):
//   r = b, x = 0;  z = V r;  p = z + beta p, beta = -(z, q_prev)/(p_prev, q_prev);
//   q = A p;  alpha = (p, r)/(p, q);  x += alpha p;  r -= alpha q.
// The scalars stay on the device; the host reads the residual norms once per
// iteration for the stopping test.
void solve_cg(Ctx &c, const double *b, double *x, int nrhs, double rtol, int maxit, cs_info *info,
              double *history, cs_status *st) {
    ensure_workspace(c, nrhs);
    Level &L0 = c.lv[0];
    const Sell &S = L0.sell;
    const int64_t n = L0.n * nrhs;
    const int64_t G = std::min<int64_t>(ceil_div(S.nslices, 4), IR_GRID);
    const int nsys = c.sys_ptr.empty() ? 1 : (int)c.sys_ptr.size() - 1;
    const bool batch = nsys > 1;
    // grown only: a release would synchronise the device (the pool waits as
    // hipFree does); a new buffer makes a captured iteration stale
    if (c.cg_r.n < (size_t)n) {
        c.cg_r.alloc(n);
        c.cg_p.alloc(n);
        c.cg_q.alloc(n);
        c.gen++;
    }
    if (c.cg_zq.n < (size_t)nsys * nrhs || c.cg_pq.n < (size_t)nsys * 2 * nrhs) {
        c.cg_zq.alloc((size_t)nsys * nrhs);
        c.cg_pq.alloc((size_t)nsys * 2 * nrhs);
        c.gen++;
    }
    double *r = c.cg_r.get(), *p = c.cg_p.get(), *q = c.cg_q.get();
    *st = CS_OK;
    const bool graphs = c.use_graphs && !c.tr.on;
    SolveStream ss(c, graphs);
    CS_HIP(hipEventRecord(c.ev0, c.stream));
    dispatch_prec(c.precision, [&](auto tp) {
        using T = std::remove_pointer_t<decltype(tp)>;
        dispatch_r(nrhs, [&](auto rc) {
            constexpr int R = decltype(rc)::value;
            T *rt = reinterpret_cast<T *>(L0.w_bb);
            const T *z = reinterpret_cast<const T *>(L0.w_xb);
            // reduce partial sums of W values per row into out[nsys][W]
            auto reduce = [&](int W, double *out) {
                if (batch)
                    hipLaunchKernelGGL(k_sys_norms, dim3(nsys), dim3(256), 0, c.stream, W, S.nrows,
                                       c.sys_ptr_d.get(), c.sys_het.get(), c.sys_spart.get(), c.rn2.get(), out);
                else
                    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(1024), 0, c.stream, G, W, c.ir_partial.get(),
                                       out);
                CS_LAUNCH_CHECK();
            };
            const double vec = (double)L0.n * R * 8.0;
            const int64_t npairs = L0.n * R / 2;
            // flat pair streaming: one system of even length, or a batch with R even
            // (pairs then never straddle two systems)
            const bool flat = batch ? R % 2 == 0 : (L0.n * R) % 2 == 0;
            int64_t Gf = G;                      // workgroups of the flat kernels
            const int32_t *sys_wg = nullptr;
            if (batch && flat) {
                std::vector<int32_t> wg(nsys + 1, 0);
                for (int q2 = 0; q2 < nsys; ++q2)
                    wg[q2 + 1] = wg[q2] + (int32_t)ceil_div((c.sys_ptr[q2 + 1] - c.sys_ptr[q2]) * R / 2, SYS_CHUNK);
                c.cg_sys_wg.upload(wg.data(), wg.size(), c.stream);
                Gf = wg[nsys];
                sys_wg = c.cg_sys_wg.get();
                if (c.cg_partial.n < (size_t)(Gf * R)) c.cg_partial.alloc(Gf * R);
            }
            double *fpart = sys_wg ? c.cg_partial.get() : c.ir_partial.get();
            auto reduce_flat = [&](double *out) {   // flat-kernel partials [Gf][R] -> out[nsys][R]
                if (sys_wg)
                    hipLaunchKernelGGL(k_wg_to_sys, dim3(nsys), dim3(256), 0, c.stream, R, sys_wg, fpart, out);
                else
                    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(1024), 0, c.stream, Gf, R, fpart, out);
                CS_LAUNCH_CHECK();
            };
            // ||b||^2 and rt = b; r = b; x = 0
            if (batch)
                hipLaunchKernelGGL((k_ir_residual<T, R, true>), dim3(G), dim3(WG), 0, c.stream, S.nrows, S.nslices,
                                   S.slice_ptr.get(), S.slice_len.get(), S.col.get(), S.val64.get(), b, nullptr, rt,
                                   (double *)nullptr, c.sys_het.get(), c.sys_spart.get(), c.rn2.get());
            else
                hipLaunchKernelGGL((k_ir_residual<T, R, false>), dim3(G), dim3(WG), 0, c.stream, S.nrows, S.nslices,
                                   S.slice_ptr.get(), S.slice_len.get(), S.col.get(), S.val64.get(), b, nullptr, rt,
                                   c.ir_partial.get(), (const int32_t *)nullptr, (double *)nullptr,
                                   (double *)nullptr);
            CS_LAUNCH_CHECK();
            reduce(R, c.ir_norm.get() + nsys * R);
            CS_HIP(hipMemcpyAsync(c.ir_norm.get(), c.ir_norm.get() + nsys * R, nsys * R * sizeof(double),
                                  hipMemcpyDeviceToDevice, c.stream));
            CS_HIP(hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
            hipLaunchKernelGGL(k_zero<double>, dim3(grid_for(n)), dim3(WG), 0, c.stream, n, x);
            CS_LAUNCH_CHECK();
            Monitor mon(c, nsys, R, rtol);
            int it = 0;
            if (!c.ev_norm) CS_HIP(hipEventCreateWithFlags(&c.ev_norm, hipEventDisableTiming));
            SpecReset spec_reset{c};
            // (p_prev, q_prev) is read by the direction update before this
            // iteration's (p, q) overwrites it: one buffer serves both
            double *pq = c.cg_pq.get();
            // one CG iteration after the check (first: p = z, no projection)
            auto iteration = [&](bool first) {
                vcycle_level<T, R>(c, 0);   // z = V r
                int slot = trace_begin(c, CS_TRACE_REFINE, first ? 0.0 : vec + L0.n * R * sizeof(T));
                if (!first) {
                    if (flat) {
                        hipLaunchKernelGGL((k_cg_zq_flat<T, R>), dim3(Gf), dim3(WG), 0, c.stream, npairs, nsys, sys_wg,
                                           c.sys_ptr_d.get(), z, q, fpart);
                        CS_LAUNCH_CHECK();
                        reduce_flat(c.cg_zq.get());
                    } else {
                        if (batch)
                            hipLaunchKernelGGL((k_cg_zq<T, R, true>), dim3(G), dim3(WG), 0, c.stream, S.nrows,
                                               S.nslices, z, q, c.sys_het.get(), c.sys_spart.get(), c.rn2.get(),
                                               (double *)nullptr);
                        else
                            hipLaunchKernelGGL((k_cg_zq<T, R, false>), dim3(G), dim3(WG), 0, c.stream, S.nrows,
                                               S.nslices, z, q, (const int32_t *)nullptr, (double *)nullptr,
                                               (double *)nullptr, c.ir_partial.get());
                        CS_LAUNCH_CHECK();
                        reduce(R, c.cg_zq.get());
                    }
                }
                if (!flat)
                    hipLaunchKernelGGL((k_cg_p<T, R>), dim3(grid_for(L0.n)), dim3(WG), 0, c.stream, L0.n, nsys,
                                       c.sys_ptr_d.get(), z, c.cg_zq.get(), pq, p, first ? 1 : 0);
                else
                    hipLaunchKernelGGL((k_cg_p_flat<T, R>), dim3(Gf), dim3(WG), 0, c.stream, npairs, nsys, sys_wg,
                                       c.sys_ptr_d.get(), z, c.cg_zq.get(), pq, p, first ? 1 : 0);
                CS_LAUNCH_CHECK();
                trace_end(c, slot);
                slot = trace_begin(c, CS_TRACE_REFINE, S.nnz * 12.0 + 3.0 * vec);
                if (batch)
                    dispatch_nb((int)L0.nb, [&](auto nbc) {
                        constexpr int NB = decltype(nbc)::value;
                        hipLaunchKernelGGL((k_cg_ap<R, true, NB>), dim3(G), dim3(WG), 0, c.stream, S.nrows, S.nslices,
                                           S.slice_ptr.get(), S.slice_len.get(), S.col.get(), S.val64.get(), p, r, q,
                                           c.sys_het.get(), c.sys_spart.get(), c.rn2.get(), (double *)nullptr);
                    });
                else
                    dispatch_nb((int)L0.nb, [&](auto nbc) {
                        constexpr int NB = decltype(nbc)::value;
                        hipLaunchKernelGGL((k_cg_ap<R, false, NB>), dim3(G), dim3(WG), 0, c.stream, S.nrows, S.nslices,
                                           S.slice_ptr.get(), S.slice_len.get(), S.col.get(), S.val64.get(), p, r, q,
                                           (const int32_t *)nullptr, (double *)nullptr, (double *)nullptr,
                                           c.ir_partial.get());
                    });
                CS_LAUNCH_CHECK();
                reduce(2 * R, pq);
                trace_end(c, slot);
                slot = trace_begin(c, CS_TRACE_REFINE, 6.0 * vec + L0.n * R * sizeof(T));
                if (flat) {
                    hipLaunchKernelGGL((k_cg_update_flat<T, R>), dim3(Gf), dim3(WG), 0, c.stream, npairs, nsys, sys_wg,
                                       c.sys_ptr_d.get(), pq, p, q, x, r, rt, fpart);
                    CS_LAUNCH_CHECK();
                    reduce_flat(c.ir_norm.get());
                } else {
                    if (batch)
                        hipLaunchKernelGGL((k_cg_update<T, R, true>), dim3(G), dim3(WG), 0, c.stream, S.nrows,
                                           S.nslices, nsys, c.sys_ptr_d.get(), pq, p, q, x, r, rt, c.sys_het.get(),
                                           c.sys_spart.get(), c.rn2.get(), (double *)nullptr);
                    else
                        hipLaunchKernelGGL((k_cg_update<T, R, false>), dim3(G), dim3(WG), 0, c.stream, S.nrows,
                                           S.nslices, nsys, c.sys_ptr_d.get(), pq, p, q, x, r, rt,
                                           (const int32_t *)nullptr, (double *)nullptr, (double *)nullptr,
                                           c.ir_partial.get());
                    CS_LAUNCH_CHECK();
                    reduce(R, c.ir_norm.get());
                }
                trace_end(c, slot);
            };
            const Ctx::GraphKey key{b, x, R, c.precision, 0, c.gen, 1};
            for (;; ++it) {
                CS_HIP(hipMemcpyAsync(c.h_norm, c.ir_norm.get(), 2 * nsys * R * sizeof(double),
                                      hipMemcpyDeviceToHost, c.stream));
                CS_HIP(hipEventRecord(c.ev_norm, c.stream));
                if (it < maxit) issue_first_sweep<T, R>(c);   // wasted (one sweep) when this check ends the solve
                CS_HIP(hipEventSynchronize(c.ev_norm));
                const double rel = mon.record(it, c.h_norm);
                if (std::isnan(rel)) {
                    *st = CS_ENAN;
                    break;
                }
                if (rel <= rtol) break;
                if (it == maxit) {
                    *st = CS_ENOCONV;
                    break;
                }
                if (it == 0) iteration(true);
                else run_iteration(c, graphs, key, [&]() { iteration(false); });
                c.spec_pending = false;
            }
            trace_flush(c);
            CS_HIP(hipEventRecord(c.ev1, c.stream));
            CS_HIP(hipEventSynchronize(c.ev1));
            float ms = 0;
            CS_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
            mon.finish(it, ms, info, history);
        });
    });
}

}  // namespace cs

namespace cs {

// Restarted GMRES(m) with the V-cycle as preconditioner (Sec. 3.1), FP64
// Krylov vectors, the V-cycle in the working precision.  Left (flexible =
// false): the Krylov space of V A and the monitored residual ||V (b - A x)||,
// the norm Sec. 3.1 regresses rho on.  Flexible (right): z_j = V v_j is kept,
// w = A z_j, x = x_0 + Z y, and the monitored residual is ||b - A x||.
// Arnoldi orthogonalises by classical Gram-Schmidt applied twice (two passes
// over the basis per step instead of j + 1); the Hessenberg columns go to the
// host, which applies Givens rotations per (system, RHS) column.  A column
// stops growing once its estimate reaches rtol ||u_0|| (or, with a left
// preconditioner in reduced precision, 1e-5 times the cycle's starting norm,
// below which the rounding of V makes the Arnoldi estimate unreliable) or on
// breakdown; the cycle ends when every column has stopped or after m steps.
// Then x is updated, the monitored residual is recomputed, and columns still
// above rtol start another cycle.
void solve_gmres(Ctx &c, const double *b, double *x, int nrhs, double rtol, int maxit, int restart, bool flexible,
                 cs_info *info, double *history, cs_status *st) {
    if (restart < 1 || restart > GM_MAXV - 1) fail(CS_EINVAL, "restart must be between 1 and 31");
    ensure_workspace(c, nrhs);
    Level &L0 = c.lv[0];
    const Sell &S = L0.sell;
    const int64_t nel = L0.n * nrhs;
    const int nsys = c.sys_ptr.empty() ? 1 : (int)c.sys_ptr.size() - 1;
    const bool batch = nsys > 1;
    const int ncol = nsys * nrhs;
    const int m = restart;
    const double inner = (!flexible && c.precision != CS_FP64) ? 1e-5 : 0.0;
    if (c.gm_V.n < (size_t)((m + 1) * nel)) c.gm_V.alloc((m + 1) * nel);
    if (flexible && c.gm_Z.n < (size_t)(m * nel)) c.gm_Z.alloc(m * nel);
    if (c.gm_w.n < (size_t)(2 * nel)) c.gm_w.alloc(2 * nel);
    c.gm_sc.alloc((size_t)(m + 1) * ncol);
    c.gm_h.alloc((size_t)(2 * (m + 1) + 1) * ncol);
    c.gm_y.alloc((size_t)ncol * m);
    int64_t Gp = std::min<int64_t>(std::max<int64_t>(ceil_div(nel, 4 * WG), 1), IR_GRID);
    const int32_t *sys_wg = nullptr;
    if (batch) {
        std::vector<int32_t> wg(nsys + 1, 0);
        for (int q = 0; q < nsys; ++q)
            wg[q + 1] = wg[q] + (int32_t)std::max<int64_t>(ceil_div((c.sys_ptr[q + 1] - c.sys_ptr[q]) * nrhs, GM_CHUNK), 1);
        c.gm_sys_wg.upload(wg.data(), wg.size(), c.stream);
        Gp = wg[nsys];
        sys_wg = c.gm_sys_wg.get();
    }
    if (c.gm_partial.n < (size_t)(Gp * (m + 1) * nrhs)) c.gm_partial.alloc(Gp * (m + 1) * nrhs);
    const size_t hcap = (size_t)(2 * (m + 1) + 1) * ncol;
    if (hcap > c.gm_host_cap) {
        if (c.gm_host) CS_HIP(hipHostFree(c.gm_host));
        c.gm_host = nullptr;
        c.gm_host_cap = 0;
        CS_HIP(hipHostMalloc(reinterpret_cast<void **>(&c.gm_host), hcap * sizeof(double)));
        c.gm_host_cap = hcap;
    }
    double *V = c.gm_V.get(), *Z = flexible ? c.gm_Z.get() : nullptr;
    double *w1 = c.gm_w.get(), *w2 = c.gm_w.get() + nel;
    double *sc = c.gm_sc.get(), *dh = c.gm_h.get(), *part = c.gm_partial.get();
    const int64_t *sysp = c.sys_ptr_d.get();
    const int64_t G = std::min<int64_t>(ceil_div(S.nslices, 4), IR_GRID);
    *st = CS_OK;
    CS_HIP(hipEventRecord(c.ev0, c.stream));
    dispatch_prec(c.precision, [&](auto tp) {
        using T = std::remove_pointer_t<decltype(tp)>;
        dispatch_r(nrhs, [&](auto rc) {
            constexpr int R = decltype(rc)::value;
            T *bb = reinterpret_cast<T *>(L0.w_bb);
            const T *xb = reinterpret_cast<const T *>(L0.w_xb);
            auto reduce = [&](int W, double *out) {
                hipLaunchKernelGGL(k_gm_reduce, dim3((unsigned)ceil_div(W, 64), (unsigned)nsys), dim3(1024), 0,
                                   c.stream, W, Gp, sys_wg, part, out);
                CS_LAUNCH_CHECK();
            };
            const dim3 gg((unsigned)Gp);
            // monitored residual u of the current x into basis slot 0, its squared
            // norms into n2 and sc_0 = 1 / ||u||
            auto monitored = [&](double *n2) {
                if (!flexible) {
                    dispatch_nb((int)L0.nb, [&](auto nbc) {
                        constexpr int NB = decltype(nbc)::value;
                        hipLaunchKernelGGL((k_gm_spmv<T, R, NB>), dim3(G), dim3(WG), 0, c.stream, S.nrows, S.nslices,
                                           S.slice_ptr.get(), S.slice_len.get(), S.col.get(), S.val64.get(), x, b,
                                           (const double *)nullptr, nsys, sysp, bb);
                    });
                    CS_LAUNCH_CHECK();
                    vcycle_level<T, R>(c, 0);
                    dispatch_mv(0, [&](auto mvc) {
                        constexpr int MV = decltype(mvc)::value;
                        hipLaunchKernelGGL((k_gm_update<T, R, false, MV>), gg, dim3(WG), 0, c.stream, nel, nsys, sys_wg, sysp,
                                           0, V, nel, sc, dh, xb, V, part);
                    });
                } else {
                    dispatch_nb((int)L0.nb, [&](auto nbc) {
                        constexpr int NB = decltype(nbc)::value;
                        hipLaunchKernelGGL((k_gm_spmv<double, R, NB>), dim3(G), dim3(WG), 0, c.stream, S.nrows, S.nslices,
                                           S.slice_ptr.get(), S.slice_len.get(), S.col.get(), S.val64.get(), x, b,
                                           (const double *)nullptr, nsys, sysp, w1);
                    });
                    dispatch_mv(0, [&](auto mvc) {
                        constexpr int MV = decltype(mvc)::value;
                        hipLaunchKernelGGL((k_gm_update<double, R, false, MV>), gg, dim3(WG), 0, c.stream, nel, nsys, sys_wg,
                                           sysp, 0, V, nel, sc, dh, (const double *)w1, V, part);
                    });
                }
                CS_LAUNCH_CHECK();
                reduce(R, n2);
                hipLaunchKernelGGL(k_gm_rscale, dim3((unsigned)ceil_div(ncol, 256)), dim3(256), 0, c.stream, ncol,
                                   n2, sc);
                CS_LAUNCH_CHECK();
                CS_HIP(hipMemcpyAsync(c.gm_host, n2, ncol * sizeof(double), hipMemcpyDeviceToHost, c.stream));
                CS_HIP(hipStreamSynchronize(c.stream));
            };
            hipLaunchKernelGGL(k_zero<double>, dim3(grid_for(nel)), dim3(WG), 0, c.stream, nel, x);
            CS_LAUNCH_CHECK();
            monitored(dh);
            std::vector<double> res(ncol), beta0(ncol), hn(2 * (size_t)ncol);
            for (int q = 0; q < ncol; ++q) {
                res[q] = std::sqrt(std::max(c.gm_host[q], 0.0));
                beta0[q] = res[q] > 0 ? res[q] : 1.0;
                hn[q] = res[q] * res[q];
                hn[ncol + q] = beta0[q] * beta0[q];
            }
            Monitor mon(c, nsys, R, rtol);
            int it = 0;
            double rel = mon.record(0, hn.data());
            std::vector<char> done(ncol);
            for (int q = 0; q < ncol; ++q) done[q] = res[q] <= rtol * beta0[q];
            // per column: Hessenberg (rotated in place), rotations, rhs g
            std::vector<double> H((size_t)ncol * (m + 1) * m), cs_(ncol * (size_t)m), sn_(ncol * (size_t)m),
                g(ncol * (size_t)(m + 1)), est(ncol), start(ncol), y((size_t)ncol * m);
            std::vector<int> steps(ncol);
            std::vector<char> growing(ncol);
            auto Hc = [&](int q, int i, int j) -> double & { return H[((size_t)q * (m + 1) + i) * m + j]; };
            while (!std::isnan(rel)) {
                bool all_done = true;
                for (int q = 0; q < ncol; ++q) all_done &= done[q] != 0;
                if (all_done) break;
                if (it == maxit) {
                    *st = CS_ENOCONV;
                    break;
                }
                for (int q = 0; q < ncol; ++q) {
                    start[q] = res[q];
                    est[q] = res[q];
                    steps[q] = 0;
                    growing[q] = !done[q];
                    std::fill(&g[(size_t)q * (m + 1)], &g[(size_t)q * (m + 1)] + m + 1, 0.0);
                    g[(size_t)q * (m + 1)] = res[q];
                }
                int j = 0;
                for (; j < m && it < maxit; ++j) {
                    const int nv = j + 1;
                    double *h1 = dh, *h2 = dh + (size_t)nv * ncol, *n2 = dh + (size_t)2 * nv * ncol;
                    double *vj = V + (int64_t)j * nel, *vn = V + (int64_t)(j + 1) * nel;
                    int slot = trace_begin(c, CS_TRACE_REFINE, S.nnz * 12.0 + (double)nel * (8.0 + sizeof(T)));
                    if (!flexible) {
                        dispatch_nb((int)L0.nb, [&](auto nbc) {
                            constexpr int NB = decltype(nbc)::value;
                            hipLaunchKernelGGL((k_gm_spmv<T, R, NB>), dim3(G), dim3(WG), 0, c.stream, S.nrows, S.nslices,
                                               S.slice_ptr.get(), S.slice_len.get(), S.col.get(), S.val64.get(), vj,
                                               (const double *)nullptr, sc + (int64_t)j * ncol, nsys, sysp, bb);
                        });
                        CS_LAUNCH_CHECK();
                        trace_end(c, slot);
                        vcycle_level<T, R>(c, 0);
                    } else {
                        hipLaunchKernelGGL((k_gm_scale_cast<T, R>), gg, dim3(WG), 0, c.stream, nel, nsys, sys_wg,
                                           sysp, vj, sc + (int64_t)j * ncol, bb);
                        CS_LAUNCH_CHECK();
                        trace_end(c, slot);
                        vcycle_level<T, R>(c, 0);
                        slot = trace_begin(c, CS_TRACE_REFINE, S.nnz * 12.0 + (double)nel * (16.0 + sizeof(T)));
                        double *zj = Z + (int64_t)j * nel;
                        hipLaunchKernelGGL((k_convert<T, double>), dim3(grid_for(nel)), dim3(WG), 0, c.stream, nel,
                                           xb, zj);
                        dispatch_nb((int)L0.nb, [&](auto nbc) {
                            constexpr int NB = decltype(nbc)::value;
                            hipLaunchKernelGGL((k_gm_spmv<double, R, NB>), dim3(G), dim3(WG), 0, c.stream, S.nrows,
                                               S.nslices, S.slice_ptr.get(), S.slice_len.get(), S.col.get(),
                                               S.val64.get(), zj, (const double *)nullptr, (const double *)nullptr, nsys,
                                               sysp, w2);
                        });
                        CS_LAUNCH_CHECK();
                        trace_end(c, slot);
                    }
                    // two Gram-Schmidt passes: h1 = V^T w, w1 = w - V h1; h2 = V^T w1, v_{j+1} = w1 - V h2
                    slot = trace_begin(c, CS_TRACE_REFINE, (3.0 * nv + 4.0) * nel * 8.0);
                    if (!flexible) {
                        dispatch_mv(nv, [&](auto mvc) {
                            constexpr int MV = decltype(mvc)::value;
                            hipLaunchKernelGGL((k_gm_dots<T, R, MV>), gg, dim3(WG), 0, c.stream, nel, nsys, sys_wg, sysp, nv,
                                               V, nel, sc, xb, part);
                        });
                        CS_LAUNCH_CHECK();
                        reduce(nv * R, h1);
                        dispatch_mv(nv, [&](auto mvc) {
                            constexpr int MV = decltype(mvc)::value;
                            hipLaunchKernelGGL((k_gm_update<T, R, true, MV>), gg, dim3(WG), 0, c.stream, nel, nsys, sys_wg,
                                               sysp, nv, V, nel, sc, h1, xb, w1, part);
                        });
                    } else {
                        dispatch_mv(nv, [&](auto mvc) {
                            constexpr int MV = decltype(mvc)::value;
                            hipLaunchKernelGGL((k_gm_dots<double, R, MV>), gg, dim3(WG), 0, c.stream, nel, nsys, sys_wg,
                                               sysp, nv, V, nel, sc, (const double *)w2, part);
                        });
                        CS_LAUNCH_CHECK();
                        reduce(nv * R, h1);
                        dispatch_mv(nv, [&](auto mvc) {
                            constexpr int MV = decltype(mvc)::value;
                            hipLaunchKernelGGL((k_gm_update<double, R, true, MV>), gg, dim3(WG), 0, c.stream, nel, nsys,
                                               sys_wg, sysp, nv, V, nel, sc, h1, (const double *)w2, w1, part);
                        });
                    }
                    CS_LAUNCH_CHECK();
                    reduce(nv * R, h2);
                    dispatch_mv(nv, [&](auto mvc) {
                        constexpr int MV = decltype(mvc)::value;
                        hipLaunchKernelGGL((k_gm_update<double, R, false, MV>), gg, dim3(WG), 0, c.stream, nel, nsys, sys_wg,
                                           sysp, nv, V, nel, sc, h2, (const double *)w1, vn, part);
                    });
                    CS_LAUNCH_CHECK();
                    reduce(R, n2);
                    hipLaunchKernelGGL(k_gm_rscale, dim3((unsigned)ceil_div(ncol, 256)), dim3(256), 0, c.stream, ncol,
                                       n2, sc + (int64_t)(j + 1) * ncol);
                    CS_LAUNCH_CHECK();
                    CS_HIP(hipMemcpyAsync(c.gm_host, dh, (size_t)(2 * nv + 1) * ncol * sizeof(double),
                                          hipMemcpyDeviceToHost, c.stream));
                    CS_HIP(hipStreamSynchronize(c.stream));
                    trace_end(c, slot);
                    ++it;
                    const double *hh1 = c.gm_host, *hh2 = c.gm_host + (size_t)nv * ncol,
                                 *hn2 = c.gm_host + (size_t)2 * nv * ncol;
                    bool any = false;
                    for (int q = 0; q < ncol; ++q) {
                        if (!growing[q]) continue;
                        const int s = q / R, k = q % R;
                        for (int i = 0; i < nv; ++i)
                            Hc(q, i, j) = hh1[((size_t)s * nv + i) * R + k] + hh2[((size_t)s * nv + i) * R + k];
                        const double hnext = std::sqrt(std::max(hn2[q], 0.0));
                        // previous rotations, then the one that annihilates H(j+1, j)
                        for (int i = 0; i < j; ++i) {
                            const double a = Hc(q, i, j), bq = Hc(q, i + 1, j);
                            Hc(q, i, j) = cs_[q * (size_t)m + i] * a + sn_[q * (size_t)m + i] * bq;
                            Hc(q, i + 1, j) = -sn_[q * (size_t)m + i] * a + cs_[q * (size_t)m + i] * bq;
                        }
                        const double a = Hc(q, j, j);
                        const double r = std::hypot(a, hnext);
                        const double cj = r > 0 ? a / r : 1.0, sj = r > 0 ? hnext / r : 0.0;
                        cs_[q * (size_t)m + j] = cj;
                        sn_[q * (size_t)m + j] = sj;
                        Hc(q, j, j) = r;
                        Hc(q, j + 1, j) = 0.0;
                        double *gq = &g[(size_t)q * (m + 1)];
                        gq[j + 1] = -sj * gq[j];
                        gq[j] = cj * gq[j];
                        est[q] = std::fabs(gq[j + 1]);
                        steps[q] = j + 1;
                        if (!(est[q] > std::max(rtol * beta0[q], inner * start[q])) || !(hnext > 0.0))
                            growing[q] = 0;
                        any |= growing[q] != 0;
                    }
                    for (int q = 0; q < ncol; ++q) hn[q] = est[q] * est[q];
                    rel = mon.record(it, hn.data());
                    if (std::isnan(rel) || !any) {
                        ++j;
                        break;
                    }
                }
                if (std::isnan(rel)) break;
                // y from the rotated triangle, x += basis y
                int kmax = 0;
                std::fill(y.begin(), y.end(), 0.0);
                for (int q = 0; q < ncol; ++q) {
                    if (done[q]) continue;
                    const int kq = steps[q];
                    kmax = std::max(kmax, kq);
                    for (int i = kq - 1; i >= 0; --i) {
                        double v = g[(size_t)q * (m + 1) + i];
                        for (int l = i + 1; l < kq; ++l) v -= Hc(q, i, l) * y[(size_t)q * m + l];
                        const double d = Hc(q, i, i);
                        y[(size_t)q * m + i] = d != 0.0 ? v / d : 0.0;
                    }
                }
                if (kmax > 0) {
                    c.gm_y.upload(y.data(), y.size(), c.stream);
                    if (!flexible)
                        dispatch_mv(kmax, [&](auto mvc) {
                            constexpr int MV = decltype(mvc)::value;
                            hipLaunchKernelGGL((k_gm_xupdate<double, R, MV>), gg, dim3(WG), 0, c.stream, nel, nsys, sys_wg,
                                               sysp, kmax, (const double *)V, nel, (const double *)sc,
                                               (const double *)c.gm_y.get(), m, x);
                        });
                    else
                        dispatch_mv(kmax, [&](auto mvc) {
                            constexpr int MV = decltype(mvc)::value;
                            hipLaunchKernelGGL((k_gm_xupdate<double, R, MV>), gg, dim3(WG), 0, c.stream, nel, nsys, sys_wg,
                                               sysp, kmax, (const double *)Z, nel, (const double *)nullptr,
                                               (const double *)c.gm_y.get(), m, x);
                        });
                    CS_LAUNCH_CHECK();
                }
                // the monitored residual of the new x replaces the last estimate
                monitored(dh);
                for (int q = 0; q < ncol; ++q) {
                    res[q] = std::sqrt(std::max(c.gm_host[q], 0.0));
                    if (!std::isfinite(c.gm_host[q])) res[q] = NAN;
                    hn[q] = res[q] * res[q];
                    done[q] = res[q] <= rtol * beta0[q];
                }
                mon.hist.pop_back();
                rel = mon.record(it, hn.data());
            }
            if (std::isnan(rel)) *st = CS_ENAN;
            trace_flush(c);
            CS_HIP(hipEventRecord(c.ev1, c.stream));
            CS_HIP(hipEventSynchronize(c.ev1));
            float ms = 0;
            CS_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
            mon.finish(it, ms, info, history);
        });
    });
}

}  // namespace cs
