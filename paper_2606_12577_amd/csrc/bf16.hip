// BF16 block kernels for 16x16 blocks (tensor Q3 DG elements): the
// multicoloured cascade sweep with A and Lambda stored in BF16 and applied on
// the matrix cores (v_mfma_f32_16x16x16bf16) with FP32 accumulation; vectors
// FP32.
//
// A block product y = M v (16x16 times a 16-vector) is one MFMA whose B
// operand holds v in every column: lane l supplies M[l%16][4(l/16)+t] and
// v[4(l/16)+t] (t = 0..3) and receives y[4(l/16)+r] (r = 0..3) in every
// column.  The received rows are exactly the k-slots a lane supplies as a B
// operand, so a residual computed by one MFMA feeds the Lambda product of the
// next without data movement.  FP32 vectors enter as a BF16 pair hi + lo
// (hi = bf16(v), lo = bf16(v - hi)): two MFMAs per block carry v to about 16
// significant bits, leaving the BF16 rounding of A and Lambda as the only
// reduced-precision step.
//
// Blocks are stored in that operand order: entry (i, k) of a block sits at
// 4 (i + 16 (k/4)) + k%4, so every lane reads its four values as one 8-byte
// load and a wavefront reads a block as one contiguous 512-byte segment.
#include <algorithm>

#include <hip/hip_ext.h>

#include "cs_internal.h"

namespace cs {
namespace {

constexpr int WG = 256;
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ void split(const float (&v)[4], bf16x4 &hi, bf16x4 &lo) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const unsigned short h = f2bf(v[t]);
        hi[t] = (short)h;
        lo[t] = (short)f2bf(v[t] - bf2f(h));
    }
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// acc + sum over the blocks [e0, e1) of a row of A_ij x_j (rows 4 kg .. 4 kg + 3).
// Blocks are taken four at a time: their block and x loads are all issued
// before the first MFMA (a wavefront then waits once per four blocks instead
// of once per block); the products are summed in block order.
__device__ __forceinline__ f32x4 block_row_product(int e0, int e1, int lane, const int32_t *__restrict__ bcol,
                                                   const unsigned short *__restrict__ aval,
                                                   const float *__restrict__ x, f32x4 acc) {
    constexpr int CH = 4;
    const int kg = lane >> 4;
    for (int e = e0; e < e1; e += CH) {
        bf16x4 a[CH];
        float4 xv[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (e + c < e1) {   // uniform per wavefront
                const int64_t j = bcol[e + c];
                a[c] = *reinterpret_cast<const bf16x4 *>(aval + (int64_t)(e + c) * 256 + lane * 4);
                xv[c] = *reinterpret_cast<const float4 *>(x + j * 16 + kg * 4);
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (e + c < e1) {
                const float v[4] = {xv[c].x, xv[c].y, xv[c].z, xv[c].w};
                bf16x4 hi, lo;
                split(v, hi, lo);
                acc = mfma(a[c], hi, acc);
                acc = mfma(a[c], lo, acc);
            }
        }
    }
    return acc;
}

// The row's first META_COLS blocks, whose block columns the row record holds:
// their block and x loads all go out at once, before the first MFMA; the
// products are summed in block order, as block_row_product does.
constexpr int META_COLS = 5;
__device__ __forceinline__ f32x4 block_row_head(int e0, int ne, const int (&col)[META_COLS], int lane,
                                                const unsigned short *__restrict__ aval,
                                                const float *__restrict__ x) {
    const int kg = lane >> 4;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    bf16x4 a[META_COLS];
    float4 xv[META_COLS];
#pragma unroll
    for (int c = 0; c < META_COLS; ++c) {
        if (c < ne) {   // uniform per wavefront
            a[c] = *reinterpret_cast<const bf16x4 *>(aval + (int64_t)(e0 + c) * 256 + lane * 4);
            xv[c] = *reinterpret_cast<const float4 *>(x + (int64_t)col[c] * 16 + kg * 4);
        }
    }
#pragma unroll
    for (int c = 0; c < META_COLS; ++c) {
        if (c < ne) {
            const float v[4] = {xv[c].x, xv[c].y, xv[c].z, xv[c].w};
            bf16x4 hi, lo;
            split(v, hi, lo);
            acc = mfma(a[c], hi, acc);
            acc = mfma(a[c], lo, acc);
        }
    }
    return acc;
}

// Multiplicative cascade step on one colour's nblk active block rows:
// x_i <- x_i - Lambda_i (sum_j A_ij x_j - b_i), in place; ZERO: x = 0 before
// the step, so x_i = Lambda_i b_i.  One wavefront per block row, read from a
// 32-byte record {row, first block, end block, c0 | c1, c2, c3, c4} that also
// holds the block columns of the row's first five blocks (the rest come from
// bcol): the x gathers of a row then wait on one load instead of two
// dependent ones.  (The 16-byte record without the columns replaced the
// colour list and the block-row pointers: 16.1 -> 15.6 us per finest-level
// colour of the 256^2 SIPG problem; two rows per wavefront with their loads
// interleaved measured 22 us.)
template <bool ZERO>
__global__ __launch_bounds__(WG) void k_bsr16_sweep(int64_t nblk, const int4 *__restrict__ meta,
                                                    const int32_t *__restrict__ bcol,
                                                    const unsigned short *__restrict__ aval,
                                                    const unsigned short *__restrict__ lam,
                                                    const float *__restrict__ b, float *x) {
    const int lane = threadIdx.x & 63, kg = lane >> 4;
    const int64_t w = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    if (w >= nblk) return;   // whole wavefront
    const int4 m = meta[2 * w];
    const int4 m2 = meta[2 * w + 1];
    const int i = m.x;
    // b and Lambda_i do not depend on the product: their loads go out first
    const float4 bv = *reinterpret_cast<const float4 *>(b + (int64_t)i * 16 + kg * 4);
    const bf16x4 l = *reinterpret_cast<const bf16x4 *>(lam + (int64_t)i * 256 + lane * 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (!ZERO) {
        const int col[META_COLS] = {m.w, m2.x, m2.y, m2.z, m2.w};
        const int ne = m.z - m.y;
        acc = block_row_head(m.y, ne < META_COLS ? ne : META_COLS, col, lane, aval, x);
        if (ne > META_COLS)   // uniform per wavefront
            acc = block_row_product(m.y + META_COLS, m.z, lane, bcol, aval, x, acc);
    }
    const float r[4] = {acc[0] - bv.x, acc[1] - bv.y, acc[2] - bv.z, acc[3] - bv.w};
    bf16x4 hi, lo;
    split(r, hi, lo);
    f32x4 y = {0.f, 0.f, 0.f, 0.f};
    y = mfma(l, hi, y);
    y = mfma(l, lo, y);
    if ((lane & 15) == 0) {
        float4 *xp = reinterpret_cast<float4 *>(x + (int64_t)i * 16 + kg * 4);
        float4 xo = ZERO ? float4{0.f, 0.f, 0.f, 0.f} : *xp;
        xo.x -= y[0];
        xo.y -= y[1];
        xo.z -= y[2];
        xo.w -= y[3];
        *xp = xo;
    }
}

__device__ __forceinline__ int64_t op_pos(int i, int k) { return 4 * (i + 16 * (k >> 2)) + (k & 3); }

// BF16 copy of A's 16x16 blocks in operand order (blocks of the block-CSR
// pattern bptr/bcol, zero-filled beforehand); one thread per scalar row
__global__ void k_pack_a16(int64_t n, const int32_t *__restrict__ ap, const int32_t *__restrict__ ac,
                           const double *__restrict__ av, const int32_t *__restrict__ bptr,
                           const int32_t *__restrict__ bcol, unsigned short *__restrict__ out) {
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row >= n) return;
    const int64_t I = row / 16;
    const int i = (int)(row % 16);
    for (int e = ap[row]; e < ap[row + 1]; ++e) {
        const int c = ac[e];
        int p = bptr[I];
        while (p < bptr[I + 1] - 1 && bcol[p] != c / 16) ++p;
        out[(int64_t)p * 256 + op_pos(i, c % 16)] = f2bf((float)av[e]);
    }
}

// Lambda blocks [depth][B][16][16] (FP64) -> operand order, plain and transposed
__global__ void k_pack_lam16(int64_t nblocks, const double *__restrict__ lam, unsigned short *__restrict__ out,
                             unsigned short *__restrict__ out_t) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= nblocks * 256) return;
    const int64_t blk = e / 256;
    const int i = (int)(e % 256) / 16, k = (int)(e % 16);
    const unsigned short v = f2bf((float)lam[e]);
    out[blk * 256 + op_pos(i, k)] = v;
    out_t[blk * 256 + op_pos(k, i)] = v;
}

__global__ void k_zero16(int64_t n, unsigned short *__restrict__ a) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) a[e] = 0;
}

inline unsigned gdim(int64_t n, int wg = WG) { return (unsigned)ceil_div(n, wg); }

}  // namespace

void build_bf16_level(Ctx &c, Level &L) {
    L.bsr_ptr.release();
    L.bsr_col.release();
    L.a16.release();
    L.bmeta.release();
    L.h_bsr_ptr.clear();
    if (L.nb != 16) return;
    // block-CSR pattern of A over all block rows (host, from the scalar CSR)
    const int64_t B = L.B;
    std::vector<int32_t> bp(B + 1, 0), bc;
    std::vector<int32_t> cols;
    for (int64_t I = 0; I < B; ++I) {
        cols.clear();
        for (int64_t r = I * 16; r < I * 16 + 16; ++r)
            for (int64_t e = L.h_ptr[r]; e < L.h_ptr[r + 1]; ++e) cols.push_back(L.h_col[e] / 16);
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        bc.insert(bc.end(), cols.begin(), cols.end());
        bp[I + 1] = (int32_t)bc.size();
    }
    L.bsr_ptr.upload(bp.data(), bp.size(), c.stream);
    L.h_bsr_ptr = bp;
    L.bsr_col.upload(bc.data(), bc.size(), c.stream);
    const int64_t tot = (int64_t)bc.size() * 256;
    L.a16.alloc(tot);
    hipLaunchKernelGGL(k_zero16, dim3(gdim(tot)), dim3(WG), 0, c.stream, tot, L.a16.get());
    hipLaunchKernelGGL(k_pack_a16, dim3(gdim(L.n)), dim3(WG), 0, c.stream, L.n, L.a_ptr.get(), L.a_col.get(),
                       L.a_val.get(), L.bsr_ptr.get(), L.bsr_col.get(), L.a16.get());
    CS_LAUNCH_CHECK();
    L.bsr_nnzb = (int64_t)bc.size();
    CS_HIP(hipStreamSynchronize(c.stream));
}

void build_bf16_meta(Ctx &c, Level &L, const std::vector<int32_t> &act) {
    L.bmeta.release();
    if (L.nb != 16 || L.h_bsr_ptr.empty() || act.empty()) return;
    // per row {row, first block, end block, c0 | c1, c2, c3, c4}: the block
    // columns of the row's first META_COLS blocks, -1 where the row is shorter
    std::vector<int32_t> cols(L.bsr_nnzb);
    L.bsr_col.download(cols.data(), cols.size(), c.stream);
    CS_HIP(hipStreamSynchronize(c.stream));
    std::vector<int32_t> m(8 * act.size());
    for (size_t q = 0; q < act.size(); ++q) {
        const int32_t i = act[q];
        const int32_t e0 = L.h_bsr_ptr[i], e1 = L.h_bsr_ptr[i + 1];
        m[8 * q] = i;
        m[8 * q + 1] = e0;
        m[8 * q + 2] = e1;
        for (int k = 0; k < META_COLS; ++k) m[8 * q + 3 + k] = e0 + k < e1 ? cols[e0 + k] : -1;
    }
    L.bmeta.upload(m.data(), m.size(), c.stream);
    CS_HIP(hipStreamSynchronize(c.stream));   // the host vector goes out of scope
}

void build_bf16_smoother(Ctx &c, Level &L) {
    L.lam16.release();
    L.lam16T.release();
    if (L.nb != 16 || L.depth == 0) return;
    const int64_t nbl = (int64_t)L.depth * L.B;
    L.lam16.alloc(nbl * 256);
    L.lam16T.alloc(nbl * 256);
    hipLaunchKernelGGL(k_pack_lam16, dim3(gdim(nbl * 256)), dim3(WG), 0, c.stream, nbl, L.lam64.get(), L.lam16.get(),
                       L.lam16T.get());
    CS_LAUNCH_CHECK();
}

bool use_bf16(const Ctx &c, const Level &L) {
    return c.precision == CS_BF16 && L.nb == 16 && L.a16.get() != nullptr;
}

// Algorithmic bytes of one colour sweep: the colour's share of A's BF16
// blocks (from a zero guess none), its Lambda blocks, b, x (read and written).
double bf16_sweep_bytes(const Level &L, int colour, bool zero) {
    const int64_t nblk = L.cblk_ptr[colour + 1] - L.cblk_ptr[colour];
    return (zero ? 0.0 : (double)L.bsr_nnzb * 512.0 * nblk / std::max<int64_t>(L.B, 1)) +
           nblk * (512.0 + 16 * 4 * (zero ? 2.0 : 3.0));
}

void bf16_sweep(Ctx &c, const Level &L, int ell, int colour, bool reverse, bool zero, const float *b, float *x) {
    const int64_t k0 = L.cblk_ptr[colour], nblk = L.cblk_ptr[colour + 1] - k0;
    if (nblk == 0) return;
    if (!L.bmeta.get()) fail(CS_ESTATE, "BF16 sweep without the colour layout's block records");
    const unsigned short *lam = (reverse ? L.lam16T.get() : L.lam16.get()) + (int64_t)ell * L.B * 256;
    // a sampled launch records its own start and end (no event packets around it)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    (void)trace_begin_launch(c, zero ? CS_TRACE_SWEEP_ZERO : (L.n >= (1 << 19) ? CS_TRACE_SWEEP
                                                                               : CS_TRACE_SWEEP_SMALL),
                             bf16_sweep_bytes(L, colour, zero), &ev0, &ev1);
    const int4 *meta = reinterpret_cast<const int4 *>(L.bmeta.get()) + 2 * k0;   // two int4 per row
    if (zero)
        hipExtLaunchKernelGGL(k_bsr16_sweep<true>, dim3(gdim(nblk, WG / 64)), dim3(WG), 0, c.stream, ev0, ev1, 0,
                              nblk, meta, L.bsr_col.get(), L.a16.get(), lam, b, x);
    else
        hipExtLaunchKernelGGL(k_bsr16_sweep<false>, dim3(gdim(nblk, WG / 64)), dim3(WG), 0, c.stream, ev0, ev1, 0,
                              nblk, meta, L.bsr_col.get(), L.a16.get(), lam, b, x);
    CS_LAUNCH_CHECK();
}

}  // namespace cs
