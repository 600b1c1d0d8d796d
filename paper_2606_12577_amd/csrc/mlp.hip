// Block-smoother network: FP32 GEMMs on the matrix cores (v_mfma_f32_16x16x4f32)
// with fused bias / SiLU / SiLU-derivative / output-scaling epilogues, MSE
// loss, Adam, and the Q1 block features.  See cascade_learned.h.
#include <algorithm>
#include <cmath>

#include "mlp_internal.h"

namespace cs {
namespace {

constexpr int WG = 256;
constexpr int TM = 64, TN = 64, TK = 16;   // workgroup tile; 4 wavefronts of 32x32
constexpr int64_t CHUNK = 16384;           // rows per evaluation chunk

typedef float f32x4 __attribute__((ext_vector_type(4)));

enum Epi { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_SILU = 2, EPI_DSILU = 3, EPI_AFFINE = 4 };

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + expf(-z)); }

// C(m, n) = sum_k A(m, k) B(k, n) with A(m, k) = A[ar(m)*sam + k*sak],
// B(k, n) = B[br(k)*sbk + n*sbn]; ar / br optional row maps (gathers).
// Epilogues: STORE C = acc; BIAS C = acc + bias[n]; BIAS_SILU aux = acc +
// bias[n], C = silu(aux); DSILU C = acc * silu'(aux[m][n]); AFFINE C = (acc +
// bias[n]) * scale[n] + shift[n].
// Tiles of 64x64 staged through LDS in 16-deep k slices; wavefront (wm, wn)
// owns the 32x32 quarter (wm, wn) as 2x2 MFMA 16x16 tiles.  MFMA operand
// layout (16x16x4, one block): lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and receives D[4*(l/16) + r][l%16] in register r.
template <int EPI>
__device__ __forceinline__ void epilogue(float v, int gm, int gn, float *__restrict__ C, int64_t ldc,
                                         const float *__restrict__ bias, float *__restrict__ aux, int64_t ldaux,
                                         const float *__restrict__ scale, const float *__restrict__ shift) {
    if constexpr (EPI == EPI_BIAS) {
        v += bias[gn];
    } else if constexpr (EPI == EPI_BIAS_SILU) {
        v += bias[gn];
        aux[(int64_t)gm * ldaux + gn] = v;
        v = v * sigmoidf(v);
    } else if constexpr (EPI == EPI_DSILU) {
        const float z = aux[(int64_t)gm * ldaux + gn];
        const float s = sigmoidf(z);
        v *= s * (1.0f + z * (1.0f - s));
    } else if constexpr (EPI == EPI_AFFINE) {
        v = (v + bias[gn]) * scale[gn] + shift[gn];
    }
    C[(int64_t)gm * ldc + gn] = v;
}

// Split K: workgroup z of the grid's third dimension sums k in
// [z kchunk, (z + 1) kchunk) and, with part given, stores its raw partial
// C_z(m, n) at part[(z M + m) N + n] for k_splitk to sum and finish.
template <int EPI>
__global__ __launch_bounds__(WG) void k_gemm(int M, int N, int K, const float *__restrict__ A, int64_t sam,
                                             int64_t sak, const int32_t *__restrict__ ar, const float *__restrict__ B,
                                             int64_t sbk, int64_t sbn, const int32_t *__restrict__ br,
                                             float *__restrict__ C, int64_t ldc, const float *__restrict__ bias,
                                             float *__restrict__ aux, int64_t ldaux, const float *__restrict__ scale,
                                             const float *__restrict__ shift, int kchunk, float *__restrict__ part) {
    __shared__ float As[TK][TM + 4];
    __shared__ float Bs[TK][TN + 4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bool a_kfast = sak == 1;
    const bool b_nfast = sbn == 1;
    const int kbeg = (int)blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int mm, kk;
            if (a_kfast) {
                mm = t >> 2;
                kk = ((t & 3) << 2) + e;
            } else {
                kk = t >> 4;
                mm = ((t & 15) << 2) + e;
            }
            const int gm = m0 + mm, gk = k0 + kk;
            float v = 0.f;
            if (gm < M && gk < kend) {
                const int64_t r = ar ? (int64_t)ar[gm] : (int64_t)gm;
                v = A[r * sam + (int64_t)gk * sak];
            }
            As[kk][mm] = v;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int kk, nn;
            if (b_nfast) {
                kk = t >> 4;
                nn = ((t & 15) << 2) + e;
            } else {
                nn = t >> 2;
                kk = ((t & 3) << 2) + e;
            }
            const int gk = k0 + kk, gn = n0 + nn;
            float v = 0.f;
            if (gk < kend && gn < N) {
                const int64_t r = br ? (int64_t)br[gk] : (int64_t)gk;
                v = B[r * sbk + (int64_t)gn * sbn];
            }
            Bs[kk][nn] = v;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < TK; ks += 4) {
            const int kr = ks + (lane >> 4);
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[kr][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int gn = n0 + wn * 32 + j * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                if (gm >= M || gn >= N) continue;
                if (part)
                    part[((int64_t)blockIdx.z * M + gm) * N + gn] = acc[i][j][r];
                else
                    epilogue<EPI>(acc[i][j][r], gm, gn, C, ldc, bias, aux, ldaux, scale, shift);
            }
        }
    }
}

// C(m, n) = epilogue(sum_z part_z(m, n)), z in increasing order
template <int EPI>
__global__ __launch_bounds__(WG) void k_splitk(int M, int N, int S, const float *__restrict__ part,
                                               float *__restrict__ C, int64_t ldc, const float *__restrict__ bias,
                                               float *__restrict__ aux, int64_t ldaux, const float *__restrict__ scale,
                                               const float *__restrict__ shift) {
    const int64_t e = blockIdx.x * (int64_t)WG + threadIdx.x, mn = (int64_t)M * N;
    if (e >= mn) return;
    float v = 0.f;
    for (int z = 0; z < S; ++z) v += part[z * mn + e];
    epilogue<EPI>(v, (int)(e / N), (int)(e % N), C, ldc, bias, aux, ldaux, scale, shift);
}

// dY = 2 (y - t') / (n * n_out) with t' = (T[row] - mean) / std; per-workgroup
// partial sums of (y - t')^2 (FP64).  dY may be null (evaluation only).
__global__ __launch_bounds__(WG) void k_mse(int64_t n, int n_out, const float *__restrict__ Y,
                                            const float *__restrict__ T, const int32_t *__restrict__ rows,
                                            const float *__restrict__ mean, const float *__restrict__ std,
                                            float *__restrict__ dY, float gscale, double *__restrict__ part) {
    __shared__ double red[WG];
    const int64_t e = blockIdx.x * (int64_t)WG + threadIdx.x;
    double sq = 0.0;
    if (e < n * n_out) {
        const int64_t r = e / n_out;
        const int c = (int)(e % n_out);
        const int64_t tr = rows ? (int64_t)rows[r] : r;
        const float tt = (T[tr * n_out + c] - mean[c]) / std[c];
        const float d = Y[e] - tt;
        if (dY) dY[e] = gscale * d;
        sq = (double)d * (double)d;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = WG / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[slot] (+)= sum of part[0..G) in a fixed order
__global__ __launch_bounds__(1024) void k_sum(int64_t G, const double *__restrict__ part, double *__restrict__ out,
                                              int slot, int accumulate) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < G; e += 1024) s += part[e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[slot] = accumulate ? out[slot] + red[0] : red[0];
}

// out[c] = sum_r D[r][c]
// Column sums of an n x ncols matrix (bias gradients): workgroup (x, y)
// covers 64 columns and rows [y rpb, (y + 1) rpb), its four wavefronts every
// fourth row; the four sums are added in order, then k_colsum_fin adds the
// row blocks' partials in order (with one row block, directly into out).
__global__ __launch_bounds__(WG) void k_colsum(int64_t n, int ncols, int64_t rpb, const float *__restrict__ D,
                                               float *__restrict__ out) {
    __shared__ float red[WG / 64][64];
    const int t = threadIdx.x, g = t >> 6;
    const int c = blockIdx.x * 64 + (t & 63);
    const int64_t r0 = (int64_t)blockIdx.y * rpb, r1 = min(n, r0 + rpb);
    float s = 0.f;
    if (c < ncols)
        for (int64_t r = r0 + g; r < r1; r += WG / 64) s += D[r * ncols + c];
    red[g][t & 63] = s;
    __syncthreads();
    if (g == 0 && c < ncols) {
        float v = red[0][t];
#pragma unroll
        for (int q = 1; q < WG / 64; ++q) v += red[q][t];
        out[(int64_t)blockIdx.y * ncols + c] = v;
    }
}

__global__ __launch_bounds__(WG) void k_colsum_fin(int ncols, int nblk, const float *__restrict__ part,
                                                   float *__restrict__ out) {
    const int c = blockIdx.x * WG + threadIdx.x;
    if (c >= ncols) return;
    float v = 0.f;
    for (int b = 0; b < nblk; ++b) v += part[(int64_t)b * ncols + c];
    out[c] = v;
}

__global__ void k_adam(int64_t np, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= np) return;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    p[e] -= lr * (me * c1) / (sqrtf(ve * c2) + eps);
}

// per-column mean and population deviation of T[rows] (two passes, FP64)
__global__ __launch_bounds__(WG) void k_colstats(int64_t n, int ncols, const float *__restrict__ T,
                                                 const int32_t *__restrict__ rows, float *__restrict__ mean,
                                                 float *__restrict__ std) {
    __shared__ double red[WG];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += WG) s += T[(rows ? (int64_t)rows[r] : r) * ncols + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double mu = red[0] / (double)n;
    __syncthreads();
    s = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += WG) {
        const double d = T[(rows ? (int64_t)rows[r] : r) * ncols + c] - mu;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double sd = sqrt(red[0] / (double)n);
        mean[c] = (float)mu;
        std[c] = sd > 0.0 ? (float)sd : 1.0f;
    }
}

// Q1 block features: one workgroup per 2x2x2 node block
constexpr int PATCH = 9, P3 = PATCH * PATCH * PATCH, NFEAT = 2 * P3 + 6;

__global__ __launch_bounds__(WG) void k_fe_features(int n, const double *__restrict__ lm, float *__restrict__ X) {
    __shared__ double rs[WG];
    __shared__ int rc[WG];
    const int nb = n / 2;
    const int64_t b = blockIdx.x;
    const int I = (int)(b % nb), J = (int)((b / nb) % nb), K = (int)(b / ((int64_t)nb * nb));
    auto hex = [&](int p, int &hi, int &hj, int &hk) {
        hi = 2 * I - 4 + p % PATCH;
        hj = 2 * J - 4 + (p / PATCH) % PATCH;
        hk = 2 * K - 4 + p / (PATCH * PATCH);
        return hi >= 0 && hi < n && hj >= 0 && hj < n && hk >= 0 && hk < n;
    };
    double s = 0.0;
    int cnt = 0;
    for (int p = threadIdx.x; p < P3; p += WG) {
        int hi, hj, hk;
        if (hex(p, hi, hj, hk)) {
            s += lm[((int64_t)hk * n + hj) * n + hi];
            ++cnt;
        }
    }
    rs[threadIdx.x] = s;
    rc[threadIdx.x] = cnt;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            rs[threadIdx.x] += rs[threadIdx.x + h];
            rc[threadIdx.x] += rc[threadIdx.x + h];
        }
        __syncthreads();
    }
    const double mean = rs[0] / (double)rc[0];
    float *out = X + b * NFEAT;
    for (int p = threadIdx.x; p < P3; p += WG) {
        int hi, hj, hk;
        const bool in = hex(p, hi, hj, hk);
        out[p] = in ? (float)((lm[((int64_t)hk * n + hj) * n + hi] - mean) / 3.0) : 0.0f;
        out[P3 + p] = in ? 1.0f : 0.0f;
    }
    if (threadIdx.x < 6) {
        const int q = threadIdx.x;
        const int c = q / 2 == 0 ? I : (q / 2 == 1 ? J : K);
        const int d = (q & 1) ? nb - 1 - c : c;
        out[2 * P3 + q] = (float)(d < 4 ? d : 4) / 4.0f;
    }
}

inline unsigned gdim(int64_t n, int wg = WG) { return (unsigned)ceil_div(n, wg); }

// A product with fewer than SPLIT_TILES output tiles and a long k (the
// training batch's weight gradients and layers) is split over k into up to
// 8 slices of at least 64, so that it runs on enough workgroups; the partial
// products go through m.kpart and k_splitk.
constexpr int SPLIT_TILES = 128;

template <int EPI>
void gemm(Mlp &m, hipStream_t s, int M, int N, int K, const float *A, int64_t sam, int64_t sak, const int32_t *ar,
          const float *B, int64_t sbk, int64_t sbn, const int32_t *br, float *C, int64_t ldc,
          const float *bias = nullptr, float *aux = nullptr, int64_t ldaux = 0, const float *scale = nullptr,
          const float *shift = nullptr) {
    if (M <= 0 || N <= 0) return;
    const int64_t tiles = (int64_t)gdim(N, TN) * gdim(M, TM);
    int S = 1;
    if (tiles < SPLIT_TILES && K >= 8 * TK)
        S = (int)std::min<int64_t>({8, ceil_div(2 * SPLIT_TILES, tiles), K / (4 * TK)});
    int kchunk = (int)ceil_div(ceil_div(K, S), TK) * TK;
    S = (int)ceil_div(K, kchunk);
    if (S > 1 && (int64_t)S * M * N > (int64_t)m.kpart.n) S = 1;
    if (S <= 1) {
        kchunk = std::max(K, 1);
        hipLaunchKernelGGL((k_gemm<EPI>), dim3(gdim(N, TN), gdim(M, TM), 1), dim3(WG), 0, s, M, N, K, A, sam, sak,
                           ar, B, sbk, sbn, br, C, ldc, bias, aux, ldaux, scale, shift, kchunk, (float *)nullptr);
    } else {
        hipLaunchKernelGGL((k_gemm<EPI>), dim3(gdim(N, TN), gdim(M, TM), S), dim3(WG), 0, s, M, N, K, A, sam, sak,
                           ar, B, sbk, sbn, br, C, ldc, bias, aux, ldaux, scale, shift, kchunk, m.kpart.get());
        hipLaunchKernelGGL((k_splitk<EPI>), dim3(gdim((int64_t)M * N)), dim3(WG), 0, s, M, N, S,
                           (const float *)m.kpart.get(), C, ldc, bias, aux, ldaux, scale, shift);
    }
    CS_LAUNCH_CHECK();
}

void ensure_cap(Mlp &m, int64_t rows) {
    if (rows <= m.cap) return;
    const size_t W = m.width, O = m.n_out;
    m.z1.alloc(rows * W);
    m.h1.alloc(rows * W);
    m.z2.alloc(rows * W);
    m.h2.alloc(rows * W);
    m.y.alloc(rows * O);
    m.dy.alloc(rows * O);
    m.d2.alloc(rows * W);
    m.d1.alloc(rows * W);
    m.part.alloc(gdim(rows * O));
    // split-k partials: up to 8 slices of the largest product that is split
    // (fewer than SPLIT_TILES output tiles)
    const int64_t split_rows = std::min<int64_t>(rows, (int64_t)SPLIT_TILES * TM);
    m.kpart.alloc((size_t)8 * std::max<int64_t>({split_rows * (int64_t)std::max(W, O), (int64_t)W * m.n_in,
                                                 (int64_t)W * (int64_t)W}));
    m.cap = rows;
}

void ensure_acc(Mlp &m, size_t slots) {
    if (m.acc.n < slots) m.acc.alloc(slots);
    if (m.h_acc_cap < slots) {
        if (m.h_acc) CS_HIP(hipHostFree(m.h_acc));
        m.h_acc = nullptr;
        m.h_acc_cap = 0;
        CS_HIP(hipHostMalloc(reinterpret_cast<void **>(&m.h_acc), slots * sizeof(double)));
        m.h_acc_cap = slots;
    }
}

// forward of n rows (rows: optional gather into X); hidden activations kept
void forward(Mlp &m, hipStream_t s, const float *X, const int32_t *rows, int64_t n, bool affine, float *Y) {
    const float *p = m.p.get();
    const int W = m.width, I = m.n_in, O = m.n_out;
    gemm<EPI_BIAS_SILU>(m, s, (int)n, W, I, X, I, 1, rows, p + m.off[0], 1, I, nullptr, m.h1.get(), W, p + m.off[1],
                        m.z1.get(), W);
    gemm<EPI_BIAS_SILU>(m, s, (int)n, W, W, m.h1.get(), W, 1, nullptr, p + m.off[2], 1, W, nullptr, m.h2.get(), W,
                        p + m.off[3], m.z2.get(), W);
    if (affine)
        gemm<EPI_AFFINE>(m, s, (int)n, O, W, m.h2.get(), W, 1, nullptr, p + m.off[4], 1, W, nullptr, Y, O, p + m.off[5],
                         nullptr, 0, m.std.get(), m.mean.get());
    else
        gemm<EPI_BIAS>(m, s, (int)n, O, W, m.h2.get(), W, 1, nullptr, p + m.off[4], 1, W, nullptr, Y, O, p + m.off[5]);
}

// loss partials of the current y against T[rows] into acc[slot]; dY when grad
void mse(Mlp &m, hipStream_t s, const float *T, const int32_t *rows, int64_t n, bool grad, int slot, bool accumulate) {
    const int64_t e = n * m.n_out;
    const unsigned G = gdim(e);
    hipLaunchKernelGGL(k_mse, dim3(G), dim3(WG), 0, s, n, m.n_out, m.y.get(), T, rows, m.mean.get(), m.std.get(),
                       grad ? m.dy.get() : nullptr, (float)(2.0 / (double)e), m.part.get());
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, s, (int64_t)G, m.part.get(), m.acc.get(), slot,
                       accumulate ? 1 : 0);
    CS_LAUNCH_CHECK();
}

void colsum(Mlp &m, hipStream_t s, int64_t n, int ncols, const float *D, float *out) {
    int64_t nblk = std::min<int64_t>(64, ceil_div(std::max<int64_t>(n, 1), 128));
    if (nblk * ncols > (int64_t)m.kpart.n) nblk = 1;
    const int64_t rpb = ceil_div(std::max<int64_t>(n, 1), nblk);
    const dim3 grid(gdim(ncols, 64), (unsigned)nblk);
    if (nblk == 1) {
        hipLaunchKernelGGL(k_colsum, grid, dim3(WG), 0, s, n, ncols, rpb, D, out);
    } else {
        hipLaunchKernelGGL(k_colsum, grid, dim3(WG), 0, s, n, ncols, rpb, D, m.kpart.get());
        hipLaunchKernelGGL(k_colsum_fin, dim3(gdim(ncols)), dim3(WG), 0, s, ncols, (int)nblk,
                           (const float *)m.kpart.get(), out);
    }
}

// gradient of the loss of the last forward (rows of X) into g
void backward(Mlp &m, hipStream_t s, const float *X, const int32_t *rows, int64_t n) {
    const float *p = m.p.get();
    float *g = m.g.get();
    const int W = m.width, I = m.n_in, O = m.n_out;
    const int N = (int)n;
    // layer 3: gW3 = dy^T h2, gb3 = colsum(dy), d2 = (dy W3) .* silu'(z2)
    gemm<EPI_STORE>(m, s, O, W, N, m.dy.get(), 1, O, nullptr, m.h2.get(), W, 1, nullptr, g + m.off[4], W);
    colsum(m, s, n, O, m.dy.get(), g + m.off[5]);
    gemm<EPI_DSILU>(m, s, N, W, O, m.dy.get(), O, 1, nullptr, p + m.off[4], W, 1, nullptr, m.d2.get(), W, nullptr,
                    m.z2.get(), W);
    // layer 2
    gemm<EPI_STORE>(m, s, W, W, N, m.d2.get(), 1, W, nullptr, m.h1.get(), W, 1, nullptr, g + m.off[2], W);
    colsum(m, s, n, W, m.d2.get(), g + m.off[3]);
    gemm<EPI_DSILU>(m, s, N, W, W, m.d2.get(), W, 1, nullptr, p + m.off[2], W, 1, nullptr, m.d1.get(), W, nullptr,
                    m.z1.get(), W);
    // layer 1
    gemm<EPI_STORE>(m, s, W, I, N, m.d1.get(), 1, W, nullptr, X, I, 1, rows, g + m.off[0], I);
    colsum(m, s, n, W, m.d1.get(), g + m.off[1]);
    CS_LAUNCH_CHECK();
}

}  // namespace

void mlp_predict(Mlp &m, hipStream_t s, const float *X, int64_t n, float *Y) {
    ensure_cap(m, std::min<int64_t>(std::max<int64_t>(n, 1), CHUNK));
    for (int64_t r0 = 0; r0 < n; r0 += CHUNK) {
        const int64_t nr = std::min<int64_t>(CHUNK, n - r0);
        forward(m, s, X + r0 * m.n_in, nullptr, nr, true, Y + r0 * m.n_out);
    }
}

}  // namespace cs

using cs::Mlp;

namespace {

template <class F>
cs_status mguarded(cs_mlp h, F &&f) {
    if (!h) return CS_EINVAL;
    Mlp &m = h->m;
    try {
        CS_HIP(hipSetDevice(m.device));
        f(m);
        m.err.clear();
        return CS_OK;
    } catch (const cs::Error &e) {
        m.err = e.msg;
        return e.st;
    } catch (const std::bad_alloc &) {
        m.err = "host allocation failed";
        return CS_ENOMEM;
    }
}

void mneed(bool ok, const std::string &msg) {
    if (!ok) cs::fail(CS_EINVAL, msg);
}

std::string g_create_err;

}  // namespace

extern "C" {

cs_status cs_mlp_create(cs_mlp *out, int32_t device, void *stream, int32_t n_in, int32_t width, int32_t n_out) {
    if (!out) return CS_EINVAL;
    *out = nullptr;
    if (n_in < 1 || width < 1 || n_out < 1 || n_in > (1 << 20) || width > 4096 || n_out > 4096) {
        g_create_err = "network sizes out of range";
        return CS_EINVAL;
    }
    cs_mlp h = new (std::nothrow) cs_mlp_s;
    if (!h) return CS_ENOMEM;
    Mlp &m = h->m;
    m.device = device;
    m.stream = reinterpret_cast<hipStream_t>(stream);
    m.n_in = n_in;
    m.width = width;
    m.n_out = n_out;
    const int64_t sz[6] = {(int64_t)width * n_in, width, (int64_t)width * width, width, (int64_t)n_out * width, n_out};
    m.off[0] = 0;
    for (int k = 0; k < 6; ++k) m.off[k + 1] = m.off[k] + sz[k];
    m.np = m.off[6];
    const cs_status st = mguarded(h, [&](Mlp &mm) {
        mm.p.alloc(mm.np);
        mm.g.alloc(mm.np);
        mm.m.alloc(mm.np);
        mm.v.alloc(mm.np);
        CS_HIP(hipMemsetAsync(mm.p.get(), 0, mm.p.bytes(), mm.stream));
        CS_HIP(hipMemsetAsync(mm.m.get(), 0, mm.m.bytes(), mm.stream));
        CS_HIP(hipMemsetAsync(mm.v.get(), 0, mm.v.bytes(), mm.stream));
        std::vector<float> zero(n_out, 0.0f), one(n_out, 1.0f);
        mm.mean.upload(zero.data(), n_out, mm.stream);
        mm.std.upload(one.data(), n_out, mm.stream);
        cs::ensure_acc(mm, 64);
        CS_HIP(hipStreamSynchronize(mm.stream));
    });
    if (st != CS_OK) {
        g_create_err = m.err;
        delete h;
        return st;
    }
    cs::pool_user(+1);
    *out = h;
    return CS_OK;
}

void cs_mlp_destroy(cs_mlp h) {
    if (!h) return;
    (void)hipSetDevice(h->m.device);
    if (h->m.h_acc) (void)hipHostFree(h->m.h_acc);
    delete h;
    cs::pool_user(-1);
}

const char *cs_mlp_last_error(cs_mlp h) { return h ? h->m.err.c_str() : g_create_err.c_str(); }

cs_status cs_mlp_param_count(cs_mlp h, int64_t *count) {
    return mguarded(h, [&](Mlp &m) {
        mneed(count != nullptr, "null output");
        *count = m.np;
    });
}

cs_status cs_mlp_set_params(cs_mlp h, const float *params) {
    return mguarded(h, [&](Mlp &m) {
        mneed(params != nullptr, "null parameters");
        for (int64_t e = 0; e < m.np; ++e) mneed(std::isfinite(params[e]), "parameters must be finite");
        m.p.upload(params, m.np, m.stream);
        CS_HIP(hipMemsetAsync(m.m.get(), 0, m.m.bytes(), m.stream));
        CS_HIP(hipMemsetAsync(m.v.get(), 0, m.v.bytes(), m.stream));
        m.step = 0;
        CS_HIP(hipStreamSynchronize(m.stream));
    });
}

cs_status cs_mlp_get_params(cs_mlp h, float *params) {
    return mguarded(h, [&](Mlp &m) {
        mneed(params != nullptr, "null output");
        m.p.download(params, m.np, m.stream);
        CS_HIP(hipStreamSynchronize(m.stream));
    });
}

cs_status cs_mlp_set_scaling(cs_mlp h, const float *mean, const float *std) {
    return mguarded(h, [&](Mlp &m) {
        mneed(mean && std, "null scaling");
        for (int c = 0; c < m.n_out; ++c) mneed(std[c] > 0.0f && std::isfinite(mean[c]), "std must be > 0");
        m.mean.upload(mean, m.n_out, m.stream);
        m.std.upload(std, m.n_out, m.stream);
        CS_HIP(hipStreamSynchronize(m.stream));
    });
}

cs_status cs_mlp_get_scaling(cs_mlp h, float *mean, float *std) {
    return mguarded(h, [&](Mlp &m) {
        mneed(mean && std, "null output");
        m.mean.download(mean, m.n_out, m.stream);
        m.std.download(std, m.n_out, m.stream);
        CS_HIP(hipStreamSynchronize(m.stream));
    });
}

cs_status cs_mlp_fit_scaling(cs_mlp h, const float *T, const int32_t *rows, int64_t n) {
    return mguarded(h, [&](Mlp &m) {
        mneed(T != nullptr && n > 0, "targets missing");
        hipLaunchKernelGGL(cs::k_colstats, dim3(m.n_out), dim3(cs::WG), 0, m.stream, n, m.n_out, T, rows,
                           m.mean.get(), m.std.get());
        CS_LAUNCH_CHECK();
        CS_HIP(hipStreamSynchronize(m.stream));
    });
}

cs_status cs_mlp_gradient(cs_mlp h, const float *X, const float *T, const int32_t *rows, int64_t n, float *grad,
                          double *loss) {
    return mguarded(h, [&](Mlp &m) {
        mneed(X && T && grad && loss && n > 0 && n <= (1 << 24), "bad gradient arguments");
        cs::ensure_cap(m, n);
        cs::forward(m, m.stream, X, rows, n, false, m.y.get());
        cs::mse(m, m.stream, T, rows, n, true, 0, false);
        cs::backward(m, m.stream, X, rows, n);
        m.g.download(grad, m.np, m.stream);
        CS_HIP(hipMemcpyAsync(m.h_acc, m.acc.get(), sizeof(double), hipMemcpyDeviceToHost, m.stream));
        CS_HIP(hipStreamSynchronize(m.stream));
        *loss = m.h_acc[0] / (double)(n * m.n_out);
    });
}

cs_status cs_mlp_loss(cs_mlp h, const float *X, const float *T, const int32_t *rows, int64_t n, double *loss) {
    return mguarded(h, [&](Mlp &m) {
        mneed(X && T && loss && n > 0, "bad loss arguments");
        cs::ensure_cap(m, std::min<int64_t>(n, cs::CHUNK));
        for (int64_t r0 = 0; r0 < n; r0 += cs::CHUNK) {
            const int64_t nr = std::min<int64_t>(cs::CHUNK, n - r0);
            const float *Xc = rows ? X : X + r0 * m.n_in;
            const float *Tc = rows ? T : T + r0 * m.n_out;
            const int32_t *rc = rows ? rows + r0 : nullptr;
            cs::forward(m, m.stream, Xc, rc, nr, false, m.y.get());
            cs::mse(m, m.stream, Tc, rc, nr, false, 0, r0 > 0);
        }
        CS_HIP(hipMemcpyAsync(m.h_acc, m.acc.get(), sizeof(double), hipMemcpyDeviceToHost, m.stream));
        CS_HIP(hipStreamSynchronize(m.stream));
        *loss = m.h_acc[0] / ((double)n * m.n_out);
    });
}

cs_status cs_mlp_train(cs_mlp h, const float *X, const float *T, const int32_t *order, int64_t n_train,
                       int32_t epochs, int32_t batch, double lr0, double lr_min, double *epoch_loss) {
    return mguarded(h, [&](Mlp &m) {
        mneed(X && T && order && n_train > 0 && epochs >= 1 && batch >= 1 && batch <= (1 << 20), "bad training "
                                                                                                   "arguments");
        mneed(lr0 > 0 && lr_min >= 0 && lr_min <= lr0, "bad learning rates");
        cs::ensure_cap(m, std::min<int64_t>(batch, n_train));
        const int64_t steps = cs::ceil_div(n_train, batch);
        cs::ensure_acc(m, (size_t)steps);
        const int64_t total = steps * epochs;
        const double b1 = 0.9, b2 = 0.999;
        int64_t k = 0;
        for (int ep = 0; ep < epochs; ++ep) {
            const int32_t *ord = order + (int64_t)ep * n_train;
            for (int64_t st = 0; st < steps; ++st, ++k) {
                const int64_t r0 = st * batch, nr = std::min<int64_t>(batch, n_train - r0);
                cs::forward(m, m.stream, X, ord + r0, nr, false, m.y.get());
                cs::mse(m, m.stream, T, ord + r0, nr, true, (int)st, false);
                cs::backward(m, m.stream, X, ord + r0, nr);
                ++m.step;
                const double lr = lr_min + 0.5 * (lr0 - lr_min) * (1.0 + std::cos(3.14159265358979323846 * (double)k / (double)total));
                const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)m.step)));
                const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)m.step)));
                hipLaunchKernelGGL(cs::k_adam, dim3(cs::gdim(m.np)), dim3(cs::WG), 0, m.stream, m.np, m.p.get(),
                                   m.g.get(), m.m.get(), m.v.get(), (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2);
                CS_LAUNCH_CHECK();
            }
            CS_HIP(hipMemcpyAsync(m.h_acc, m.acc.get(), steps * sizeof(double), hipMemcpyDeviceToHost, m.stream));
            CS_HIP(hipStreamSynchronize(m.stream));
            double s = 0.0;
            for (int64_t st = 0; st < steps; ++st) {
                const int64_t nr = std::min<int64_t>(batch, n_train - st * batch);
                s += m.h_acc[st] / ((double)nr * m.n_out);
            }
            if (epoch_loss) epoch_loss[ep] = s / (double)steps;
            mneed(std::isfinite(s), "training diverged (non-finite loss)");
        }
    });
}

cs_status cs_mlp_forward(cs_mlp h, const float *X, int64_t n, float *Y) {
    return mguarded(h, [&](Mlp &m) {
        mneed(X && Y && n > 0, "bad forward arguments");
        cs::mlp_predict(m, m.stream, X, n, Y);
        CS_HIP(hipStreamSynchronize(m.stream));
    });
}

cs_status cs_fe_block_features(void *stream, const double *log10mu, int32_t n, float *X) {
    if (!log10mu || !X || n < 2 || n % 2 || n > 4096) return CS_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t nb = n / 2;
    hipLaunchKernelGGL(cs::k_fe_features, dim3((unsigned)(nb * nb * nb)), dim3(cs::WG), 0, s, n, log10mu, X);
    if (hipGetLastError() != hipSuccess) return CS_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return CS_EDEVICE;
    return CS_OK;
}

}  // extern "C"
