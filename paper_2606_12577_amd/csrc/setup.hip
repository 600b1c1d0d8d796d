// Setup of cascading smoothers on the GPU (gfx950, wave64).
//
// Implements, per multigrid level, the construction of Sec. 2.1-2.3:
//   prescale      W = diag(a_kk^{-1/2}), A~ = W A W            (Sec. 2.3.1)
//   symbolic      pattern(M_i) = union_{j in adj(i)} pattern(E_j)
//   row product   M_i = sum_j A~_ij E_j,:                       (Alg. 2, LS step)
//   normal eqs    G_i = M_i M_i^T, H_i = E_i M_i^T, Lambda~_i = H_i G_i^{-1}
//   update        E_i <- E_i - Lambda~_i M_i                     (Alg. 2, update)
//   truncation    keep the alpha largest blocks of a row of E   (Alg. 2, option)
//   unscale       Lambda_i = W_i Lambda~_i W_i                   (Alg. 2, last step)
// The multicoloured variant (Sec. 2.2) runs the same fit step over the blocks of
// one colour at a time, leaving the rows of the other colours untouched.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <type_traits>

#include "cs_internal.h"

namespace cs {

namespace {

constexpr int WG = 256;
constexpr int UNION_CAP = 4096;   // candidate columns per row in the symbolic step (a power of two)
constexpr int UNION_CAP_BIG = 8192;   // the same for wide rows (32 KB of LDS; a power of two: the sort pads to one)
constexpr int MATCH_CAP = 8192;   // (column, neighbour) matches cached per row
constexpr int MAXNB = 16;
constexpr double PIVOT_TOL = 1e-13;

__device__ inline int bsearch_i32(const int32_t *a, int lo, int hi, int32_t key) {
    // index of key in the sorted range a[lo, hi), or -1
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        int32_t v = a[mid];
        if (v == key) return mid;
        if (v < key) lo = mid + 1;
        else hi = mid;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// prescaling
// ---------------------------------------------------------------------------
// Elliptic prescaling (Sec. 2.3.1): w = a_kk^{-1/2}; bad[k] = 1 for a diagonal
// that is not positive.
__global__ void k_prescale_w(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                             const double *__restrict__ val, int64_t n, double *__restrict__ w,
                             int32_t *__restrict__ bad) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    double d = 0.0;
    for (int k = ptr[r]; k < ptr[r + 1]; ++k)
        if (col[k] == r) d = val[k];
    bad[r] = d > 0.0 ? 0 : 1;
    w[r] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
}

// Stokes prescaling (Sec. 2.3.2), velocity (and inert) rows: with the viscous
// block V (columns that are not pressures), w = sqrt(||V_r,:||_1) / V_rr, so
// that the prescaled diagonal is ||V_r,:||_1 / V_rr.
__global__ void k_prescale_stokes_v(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                    const double *__restrict__ val, const int32_t *__restrict__ kind, int64_t n,
                                    double *__restrict__ w, int32_t *__restrict__ bad) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n || kind[r] == 1) return;
    double d = 0.0, l1 = 0.0;
    for (int k = ptr[r]; k < ptr[r + 1]; ++k) {
        const int c = col[k];
        if (kind[c] == 1) continue;
        l1 += fabs(val[k]);
        if (c == r) d = val[k];
    }
    bad[r] = d > 0.0 ? 0 : 1;
    w[r] = d > 0.0 ? sqrt(l1) / d : 1.0;
}

// pressure rows: every row of diag(w_p) D diag(w_u) gets unit max-norm
// (l1 = 0) or unit 1-norm (l1 = 1)
__global__ void k_prescale_stokes_p(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                    const double *__restrict__ val, const int32_t *__restrict__ kind, int64_t n,
                                    int l1, double *__restrict__ w, int32_t *__restrict__ bad) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n || kind[r] != 1) return;
    double m = 0.0;
    for (int k = ptr[r]; k < ptr[r + 1]; ++k) {
        const int c = col[k];
        if (kind[c] == 1) continue;
        const double v = fabs(val[k] * w[c]);
        m = l1 ? m + v : fmax(m, v);
    }
    bad[r] = m > 0.0 ? 0 : 1;
    w[r] = m > 0.0 ? 1.0 / m : 1.0;
}

// A~ as dense nb x nb blocks on the block pattern of A.
__global__ void k_scatter_blocks(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                 const double *__restrict__ val, const double *__restrict__ w, int64_t n, int nb,
                                 const int32_t *__restrict__ bptr, const int32_t *__restrict__ bcol,
                                 double *__restrict__ bval) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    int i = (int)(r / nb), lr = (int)(r % nb);
    for (int k = ptr[r]; k < ptr[r + 1]; ++k) {
        int c = col[k];
        int pos = bsearch_i32(bcol, bptr[i], bptr[i + 1], c / nb);
        if (pos < 0) continue;  // cannot happen: the block pattern covers every entry
        bval[(int64_t)pos * nb * nb + lr * nb + (c % nb)] = val[k] * w[r] * w[c];
    }
}

// ---------------------------------------------------------------------------
// symbolic union of sorted column lists (one workgroup per output row)
// ---------------------------------------------------------------------------
// SRC_SCALAR: candidates of block row i are the block columns of the scalar
//             entries of its nb rows (the block pattern of A).
// SRC_E:      candidates are the columns of E_j for j in the block row i of A.
enum { SRC_SCALAR = 0, SRC_E = 1 };

template <int SRC, bool FILL, int CAP = UNION_CAP>
__global__ __launch_bounds__(WG) void k_union(const int32_t *__restrict__ list, int nlist, int nb,
                                              const int32_t *__restrict__ sptr, const int32_t *__restrict__ scol,
                                              const int32_t *__restrict__ eptr, const int32_t *__restrict__ ecol,
                                              int32_t *__restrict__ out_cnt, const int32_t *__restrict__ out_ptr,
                                              int32_t *__restrict__ out_col, int32_t *__restrict__ err) {
    __shared__ int32_t cand[CAP];
    __shared__ int32_t offs[257];
    __shared__ int32_t part[WG + 1];
    __shared__ int32_t total_s;
    const int li = (int)xcd_tile(blockIdx.x, gridDim.x);   // rows of a range share the XCD's L2
    if (li >= nlist) return;
    const int i = list ? list[li] : li;
    const int t = threadIdx.x;
    int total;
    if (SRC == SRC_SCALAR) {
        int lo = sptr[(int64_t)i * nb], hi = sptr[(int64_t)(i + 1) * nb];
        total = hi - lo;
        if (total > CAP) {
            if (t == 0) err[li] = 1;
            if (!FILL && t == 0) out_cnt[li] = 0;
            return;
        }
        for (int k = t; k < total; k += WG) cand[k] = scol[lo + k] / nb;
    } else {
        int lo = sptr[i], hi = sptr[i + 1];
        int deg = hi - lo;
        if (deg > 256) {
            if (t == 0) err[li] = 2;
            if (!FILL && t == 0) out_cnt[li] = 0;
            return;
        }
        if (t < deg) {
            int j = scol[lo + t];
            offs[t + 1] = eptr[j + 1] - eptr[j];
        }
        __syncthreads();
        if (t == 0) {
            offs[0] = 0;
            for (int q = 0; q < deg; ++q) offs[q + 1] += offs[q];
            total_s = offs[deg];
        }
        __syncthreads();
        total = total_s;
        if (total > CAP) {
            if (t == 0) err[li] = 1;
            if (!FILL && t == 0) out_cnt[li] = 0;
            return;
        }
        for (int k = t; k < total; k += WG) {
            int q = 0;
            while (offs[q + 1] <= k) ++q;
            int j = scol[lo + q];
            cand[k] = ecol[eptr[j] + (k - offs[q])];
        }
    }
    int P = 1;
    while (P < total) P <<= 1;
    for (int k = total + t; k < P; k += WG) cand[k] = INT32_MAX;
    __syncthreads();
    // bitonic sort of cand[0, P)
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int a = t; a < P; a += WG) {
                int b = a ^ j;
                if (b > a) {
                    int32_t x = cand[a], y = cand[b];
                    bool up = (a & k) == 0;
                    if ((x > y) == up) {
                        cand[a] = y;
                        cand[b] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    // unique: each thread owns a contiguous chunk
    const int chunk = (P + WG - 1) / WG;
    const int a0 = t * chunk, a1 = min(P, a0 + chunk);
    int mine = 0;
    for (int a = a0; a < a1; ++a) {
        int32_t v = cand[a];
        if (v != INT32_MAX && (a == 0 || cand[a - 1] != v)) ++mine;
    }
    part[t + 1] = mine;
    __syncthreads();
    if (t == 0) {
        part[0] = 0;
        for (int q = 0; q < WG; ++q) part[q + 1] += part[q];
    }
    __syncthreads();
    if (!FILL) {
        if (t == 0) out_cnt[li] = part[WG];
    } else {
        int o = out_ptr[li] + part[t];
        for (int a = a0; a < a1; ++a) {
            int32_t v = cand[a];
            if (v != INT32_MAX && (a == 0 || cand[a - 1] != v)) out_col[o++] = v;
        }
    }
}

// The same union, one wavefront per output row, for rows of at most 64 K
// candidates (and, for SRC_E, at most 64 neighbours): the candidates sit in K
// registers per lane (element e = 64 r + lane), are sorted by a bitonic network
// of register exchanges (distance >= 64) and lane shuffles (distance < 64), and
// the distinct values are compacted with ballots.  The host picks K from an
// upper bound of the candidate count; a row above it sets err (cannot happen).
template <int K, int SRC, bool FILL>
__global__ __launch_bounds__(WG) void k_union_wave(const int32_t *__restrict__ list, int nlist, int nb,
                                                   const int32_t *__restrict__ sptr,
                                                   const int32_t *__restrict__ scol,
                                                   const int32_t *__restrict__ eptr,
                                                   const int32_t *__restrict__ ecol, int32_t *__restrict__ out_cnt,
                                                   const int32_t *__restrict__ out_ptr, int32_t *__restrict__ out_col,
                                                   int32_t *__restrict__ err) {
    constexpr int P = 64 * K;
    __shared__ int32_t offs_s[WG / 64][65], start_s[WG / 64][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = (int)xcd_tile(blockIdx.x, gridDim.x) * (WG / 64) + wv;   // see k_union
    const bool live = li < nlist;
    const int i = live ? (list ? list[li] : li) : 0;
    int total = 0, lo = 0, deg = 0;
    if (SRC == SRC_SCALAR) {
        if (live) {
            lo = sptr[(int64_t)i * nb];
            total = sptr[(int64_t)(i + 1) * nb] - lo;
        }
    } else {
        if (live) {
            lo = sptr[i];
            deg = sptr[i + 1] - lo;
        }
        int len = 0;
        if (lane < deg) {
            const int j = scol[lo + lane];
            start_s[wv][lane] = eptr[j];
            len = eptr[j + 1] - eptr[j];
        }
        int inc = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        offs_s[wv][lane + 1] = inc;
        if (lane == 0) offs_s[wv][0] = 0;
        total = __shfl(inc, 63, 64);
        if (deg > 64) total = P + 1;
    }
    __syncthreads();   // every wavefront reaches it: offs_s and start_s are visible
    if (total > P) {
        if (lane == 0) {
            err[li] = 1;
            if (!FILL) out_cnt[li] = 0;
        }
        return;
    }
    int32_t v[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int e = r * 64 + lane;
        v[r] = INT32_MAX;
        if (e < total) {
            if (SRC == SRC_SCALAR) {
                v[r] = scol[lo + e] / nb;
            } else {
                int a = 0, b = deg;   // offs[a] <= e < offs[b]
                while (b - a > 1) {
                    const int m = (a + b) >> 1;
                    if (offs_s[wv][m] <= e) a = m;
                    else b = m;
                }
                v[r] = ecol[start_s[wv][a] + (e - offs_s[wv][a])];
            }
        }
    }
#pragma unroll
    for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    const int rp = r ^ (j >> 6);
                    if (rp > r) {
                        const bool up = ((r * 64 + lane) & k) == 0;
                        const int32_t x = v[r], y = v[rp];
                        if ((x > y) == up) {
                            v[r] = y;
                            v[rp] = x;
                        }
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    const int32_t y = __shfl_xor(v[r], j, 64);
                    const bool up = ((r * 64 + lane) & k) == 0;
                    const bool lower = (lane & j) == 0;
                    v[r] = (lower == up) ? min(v[r], y) : max(v[r], y);
                }
            }
        }
    }
    int base = live ? (FILL ? out_ptr[li] : 0) : 0;
    int count = 0;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        // element e - 1: lane - 1 of register r, or lane 63 of register r - 1
        const int32_t up1 = __shfl_up(v[r], 1, 64);
        const int32_t last = r > 0 ? __shfl(v[r > 0 ? r - 1 : 0], 63, 64) : INT32_MIN;
        const int32_t prev = lane == 0 ? last : up1;
        const bool keep = v[r] != INT32_MAX && prev != v[r];
        const uint64_t mask = __ballot(keep);
        if (FILL && keep) {
            const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            out_col[base + count + below] = v[r];
        }
        count += __popcll(mask);
    }
    if (!FILL && live && lane == 0) out_cnt[li] = count;
}

// Exclusive prefix sum of n counts in three passes: every workgroup scans 1024
// counts and records its total, one workgroup scans the totals, and the
// offsets are added (coalesced; the totals are exact in 64 bits).
constexpr int SCAN_TILE = 1024;

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *sh, int64_t &total) {
    // 256 threads, Hillis-Steele in LDS
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int64_t add = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    total = sh[255];
    const int64_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(256) void k_scan_tiles(const int32_t *__restrict__ cnt, int64_t n,
                                                    int32_t *__restrict__ ptr, int64_t *__restrict__ tile_sum) {
    __shared__ int64_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 4;
    int64_t v[4], local = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        v[u] = base + u < n ? cnt[base + u] : 0;
        local += v[u];
    }
    int64_t total;
    int64_t o = block_exclusive_scan(local, sh, total);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (base + u < n) ptr[base + u] = (int32_t)o;
        o += v[u];
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_sums(int64_t ntiles, int64_t *__restrict__ tile_sum,
                                                   int64_t *__restrict__ total_out) {
    __shared__ int64_t sh[256];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < ntiles; b0 += 256) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t v = b < ntiles ? tile_sum[b] : 0;
        int64_t total;
        const int64_t o = block_exclusive_scan(v, sh, total);
        if (b < ntiles) tile_sum[b] = carry + o;
        carry += total;
    }
    if (threadIdx.x == 0) total_out[0] = carry;
}

__global__ __launch_bounds__(256) void k_scan_add(int64_t n, const int64_t *__restrict__ tile_off,
                                                  const int64_t *__restrict__ total, int32_t *__restrict__ ptr) {
    const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (a < n) ptr[a] += (int32_t)tile_off[a / SCAN_TILE];
    if (a == 0) ptr[n] = (int32_t)total[0];
}

// ---------------------------------------------------------------------------
// numeric fit step
// ---------------------------------------------------------------------------

// M_i = sum_{j in adj(i)} A~_ij E_j,:  on pattern(M_i); one workgroup per list row.
__global__ __launch_bounds__(WG) void k_rowprod(const int32_t *__restrict__ list, int nb,
                                                const int32_t *__restrict__ abptr, const int32_t *__restrict__ abcol,
                                                const double *__restrict__ abval, const int32_t *__restrict__ eptr,
                                                const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                                const int32_t *__restrict__ mptr, const int32_t *__restrict__ mcol,
                                                double *__restrict__ mval) {
    __shared__ int32_t match[MATCH_CAP];
    const int li = (int)xcd_tile(blockIdx.x, gridDim.x);   // see k_rowprod_nb
    const int i = list[li];
    const int t = threadIdx.x;
    const int alo = abptr[i], deg = abptr[i + 1] - alo;
    const int mlo = mptr[li], k = mptr[li + 1] - mlo;
    const int nb2 = nb * nb;
    const bool cached = (int64_t)k * deg <= MATCH_CAP;
    if (cached) {
        for (int e = t; e < k * deg; e += WG) {
            int p = e / deg, jj = e % deg;
            int j = abcol[alo + jj];
            match[e] = bsearch_i32(ecol, eptr[j], eptr[j + 1], mcol[mlo + p]);
        }
        __syncthreads();
    }
    for (int64_t e = t; e < (int64_t)k * nb2; e += WG) {
        int p = (int)(e / nb2), rs = (int)(e % nb2);
        int r = rs / nb, s = rs % nb;
        double acc = 0.0;
        for (int jj = 0; jj < deg; ++jj) {
            int q;
            if (cached) q = match[p * deg + jj];
            else {
                int j = abcol[alo + jj];
                q = bsearch_i32(ecol, eptr[j], eptr[j + 1], mcol[mlo + p]);
            }
            if (q < 0) continue;
            const double *a = abval + (int64_t)(alo + jj) * nb2 + r * nb;
            const double *ev = eval + (int64_t)q * nb2 + s;
            for (int u = 0; u < nb; ++u) acc += a[u] * ev[u * nb];
        }
        mval[(int64_t)(mlo + p) * nb2 + rs] = acc;
    }
}

// The same product with the A~_ij blocks of the row staged in LDS and one
// thread per (block column p, column s) of M_i computing all NB rows: every
// E entry is read from memory once per (p, j) instead of NB times, and the
// A~ values come from LDS as wavefront broadcasts.
constexpr int AS_CAP = 2048;   // at most this many doubles of A~ staged per row (deg * NB^2)
constexpr int MATCH_NB = 1024; // (column, neighbour) matches cached per row
constexpr int ECOL_CAP = 1024; // column indices of the neighbours' E rows staged per row
constexpr int DEG_CAP = 32;    // neighbours whose E column lists are staged
// LDS and registers sized for eight waves per SIMD with blocks of up to 8x8:
// the staging buffer of A~ is sized at launch from the level's largest block
// row (a 7-point stencil's 7 blocks of 8x8: 3.5 KB), the rest is 8.3 KB; 62
// VGPRs.  128^3 setup 53.6 -> 50.6 ms against five waves (92 VGPRs, 32 KB).

// as_n: doubles of the dynamic LDS buffer that stages A~ (a row is staged
// when deg * NB^2 <= as_n).  WGS: threads per row (one workgroup per row); 64
// for the early steps whose short rows leave most of 256 threads idle (the
// match and column tables shrink with it, so four times the rows run per CU).
template <int NB, int WGS = WG>
__global__ __launch_bounds__(WGS, NB <= 8 ? 6 * (WG / WGS) : 1) void k_rowprod_nb(const int32_t *__restrict__ list,
                                                                    const int32_t *__restrict__ abptr,
                                                                    const int32_t *__restrict__ abcol,
                                                                    const double *__restrict__ abval,
                                                                    const int32_t *__restrict__ eptr,
                                                                    const int32_t *__restrict__ ecol,
                                                                    const double *__restrict__ eval,
                                                                    const int32_t *__restrict__ mptr,
                                                                    const int32_t *__restrict__ mcol,
                                                                    double *__restrict__ mval, int as_n) {
    constexpr int NB2 = NB * NB;
    constexpr int MATCH_W = MATCH_NB * WGS / WG, ECOL_W = ECOL_CAP * WGS / WG;
    __shared__ int32_t match[MATCH_W];
    extern __shared__ __align__(16) double As[];
    // consecutive rows on one XCD: the E_j rows gathered by a row are gathered
    // again by its neighbours, which then find them in that XCD's L2 (with the
    // hardware's round-robin order neighbours ran on different XCDs; the
    // 128^3 problem's largest launch fetched 44.5 GB against 8.5 GB of E)
    const int li = (int)xcd_tile(blockIdx.x, gridDim.x);
    const int i = list[li];
    const int t = threadIdx.x;
    const int alo = abptr[i], deg = abptr[i + 1] - alo;
    const int mlo = mptr[li], k = mptr[li + 1] - mlo;
    const bool cached = (int64_t)k * deg <= MATCH_W;   // uniform per workgroup
    const bool staged = deg * NB2 <= as_n;
    // staged blocks are stored transposed (column u of A~_ij contiguous), so one
    // 16-byte LDS read feeds two rows of the product
    if (staged)
        for (int e = t; e < deg * NB2; e += WGS) {
            const int jj = e / NB2, rs = e % NB2;
            As[jj * NB2 + (rs % NB) * NB + rs / NB] = abval[(int64_t)alo * NB2 + e];
        }
    // The neighbours' E column lists, concatenated in LDS with one coalesced
    // read, so that the k * deg searches of the matches run in LDS instead of
    // as chains of dependent global loads (the same positions either way).
    __shared__ int32_t ecs[ECOL_W];
    __shared__ int32_t eoff[DEG_CAP + 1], elo_s[DEG_CAP];
    bool ecols = false;   // uniform
    if (cached && deg <= DEG_CAP) {
        if (t < deg) {
            const int j = abcol[alo + t];
            elo_s[t] = eptr[j];
            eoff[t + 1] = eptr[j + 1] - eptr[j];
        }
        if (t == 0) eoff[0] = 0;
        __syncthreads();
        if (t == 0)
            for (int jj = 0; jj < deg; ++jj) eoff[jj + 1] += eoff[jj];
        __syncthreads();
        const int tot = eoff[deg];
        ecols = tot <= ECOL_W;
        if (ecols)
            for (int e = t; e < tot; e += WGS) {
                int jj = 0;
                while (eoff[jj + 1] <= e) ++jj;
                ecs[e] = ecol[elo_s[jj] + e - eoff[jj]];
            }
        __syncthreads();
    }
    if (cached)
        for (int e = t; e < k * deg; e += WGS) {
            const int p = e / deg, jj = e % deg;
            if (ecols) {
                const int r = bsearch_i32(ecs, eoff[jj], eoff[jj + 1], mcol[mlo + p]);
                match[e] = r < 0 ? -1 : elo_s[jj] + (r - eoff[jj]);
            } else {
                const int j = abcol[alo + jj];
                match[e] = bsearch_i32(ecol, eptr[j], eptr[j + 1], mcol[mlo + p]);
            }
        }
    __syncthreads();
    if constexpr (NB % 2 == 0) {
        if (staged) {   // two adjacent columns of M per thread (same summation order per entry)
            constexpr int NH = NB / 2;
            for (int w = t; w < k * NH; w += WGS) {
                const int p = w / NH, c2 = (w % NH) * 2;
                double a0[NB], a1[NB];
#pragma unroll
                for (int r = 0; r < NB; ++r) a0[r] = a1[r] = 0.0;
                for (int jj = 0; jj < deg; ++jj) {
                    int q;
                    if (cached) {
                        q = match[p * deg + jj];
                    } else {
                        const int j = abcol[alo + jj];
                        q = bsearch_i32(ecol, eptr[j], eptr[j + 1], mcol[mlo + p]);
                    }
                    if (q < 0) continue;
                    const double *ev = eval + (int64_t)q * NB2 + c2;
                    const double2 *a2 = reinterpret_cast<const double2 *>(As + jj * NB2);
                    // the NB loads of a block first (all in flight), then the products
                    double2 eb[NB];
#pragma unroll
                    for (int u = 0; u < NB; ++u) eb[u] = *reinterpret_cast<const double2 *>(ev + u * NB);
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        const double2 e = eb[u];
#pragma unroll
                        for (int r2 = 0; r2 < NH; ++r2) {
                            const double2 av = a2[u * NH + r2];
                            a0[2 * r2] += av.x * e.x;
                            a0[2 * r2 + 1] += av.y * e.x;
                            a1[2 * r2] += av.x * e.y;
                            a1[2 * r2 + 1] += av.y * e.y;
                        }
                    }
                }
                // streaming stores: M (up to 17 GB a step on the 128^3 level) is
                // read back once by the normal equations (setup 59.5 -> 58.4 ms)
                double *mo = mval + (int64_t)(mlo + p) * NB2 + c2;
                typedef double d2v __attribute__((ext_vector_type(2)));
#pragma unroll
                for (int r = 0; r < NB; ++r) {
                    const d2v v = {a0[r], a1[r]};
                    __builtin_nontemporal_store(v, reinterpret_cast<d2v *>(mo + r * NB));
                }
            }
            return;
        }
    }
    for (int w = t; w < k * NB; w += WGS) {
        const int p = w / NB, sc = w % NB;
        double acc[NB];
#pragma unroll
        for (int r = 0; r < NB; ++r) acc[r] = 0.0;
        for (int jj = 0; jj < deg; ++jj) {
            int q;
            if (cached) {
                q = match[p * deg + jj];
            } else {
                const int j = abcol[alo + jj];
                q = bsearch_i32(ecol, eptr[j], eptr[j + 1], mcol[mlo + p]);
            }
            if (q < 0) continue;
            const double *ev = eval + (int64_t)q * NB2 + sc;
            if (staged) {   // (odd NB: the even sizes returned above)
#pragma unroll 2
                for (int u = 0; u < NB; ++u) {
                    const double e = ev[u * NB];
#pragma unroll
                    for (int r = 0; r < NB; ++r) acc[r] += As[jj * NB2 + u * NB + r] * e;
                }
                continue;
            }
            const double *a = abval + (int64_t)(alo + jj) * NB2;
#pragma unroll 2
            for (int u = 0; u < NB; ++u) {
                const double e = ev[u * NB];
#pragma unroll
                for (int r = 0; r < NB; ++r) acc[r] += a[r * NB + u] * e;
            }
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) mval[(int64_t)(mlo + p) * NB2 + r * NB + sc] = acc[r];
    }
}

// Lambda~ (G + tau I) = H for one block (G, H: nb x nb in LDS, row-major), by
// the whole workgroup, tau = ridge tr(G) / nb (ridge = 0: the plain normal
// equations; ridge > 0: the Tikhonov-regularised fit).  Lc and V are LDS
// scratch of MAXNB^2 doubles.  Writes Lambda~ to out and, from thread 0,
// whether the matrix was (numerically) singular to *singular.
__device__ void normal_solve(const double *G, const double *H, double *Lc, double *V, int nb,
                             double *__restrict__ out, int32_t *__restrict__ singular, double ridge) {
    const int t = threadIdx.x;
    const int nb2 = nb * nb;
    double trace = 0.0;
    for (int q = 0; q < nb; ++q) trace += G[q * nb + q];
    const double tau = ridge > 0.0 ? ridge * trace / nb : 0.0;
    // Lambda~ G = H.  Regular G: Gauss-Jordan inverse of [G | I] (G is SPD:
    // no pivoting; the pivots are the Cholesky pivots squared, with the same
    // cut-off), one thread per entry, two barriers per step.  A pivot below
    // PIVOT_TOL max diag(G) marks G as (numerically) singular: then the
    // minimum-norm solution through a parallel cyclic Jacobi eigen-decomposition.
    __shared__ double Aug[MAXNB * 2 * MAXNB];
    const int w2 = 2 * nb;
    double dmax = 0.0;
    for (int q = 0; q < nb; ++q) dmax = fmax(dmax, G[q * nb + q] + tau);
    bool bad = !(dmax > 0.0);
    for (int e = t; e < nb * w2; e += WG) {
        const int r = e / w2, c = e % w2;
        Aug[e] = c < nb ? G[r * nb + c] + (r == c ? tau : 0.0) : (c - nb == r ? 1.0 : 0.0);
    }
    __syncthreads();
    constexpr int PER = (MAXNB * 2 * MAXNB + WG - 1) / WG;
    for (int q = 0; q < nb && !bad; ++q) {
        const double piv = Aug[q * w2 + q];
        if (!(piv > PIVOT_TOL * dmax)) {   // same value in every thread: uniform
            bad = true;
            break;
        }
        double f[PER], g[PER];
#pragma unroll
        for (int k2 = 0; k2 < PER; ++k2) {
            const int e = t + k2 * WG;
            if (e < nb * w2) {
                f[k2] = Aug[(e / w2) * w2 + q];
                g[k2] = Aug[q * w2 + e % w2];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < PER; ++k2) {
            const int e = t + k2 * WG;
            if (e < nb * w2) Aug[e] = (e / w2 == q) ? g[k2] / piv : Aug[e] - f[k2] * g[k2] / piv;
        }
        __syncthreads();
    }
    if (t == 0) *singular = bad ? 1 : 0;
    if (!bad) {
        if (t < nb2) {
            const int r = t / nb, c = t % nb;
            double acc = 0.0;
            for (int u = 0; u < nb; ++u) acc += H[r * nb + u] * Aug[u * w2 + nb + c];
            out[t] = acc;
        }
        return;
    }
    // ---- (near-)singular G: Lambda~ = H V diag(1/ev, ev kept) V^T
    const int m = nb + (nb & 1);   // even order for the round-robin pairing (zero padding)
    __shared__ int pp_s[MAXNB / 2], pq_s[MAXNB / 2], pair_of[MAXNB], side_of[MAXNB];
    __shared__ double rc_s[MAXNB / 2], rs_s[MAXNB / 2], off_s[WG], dia_s[WG];
    for (int e = t; e < m * m; e += WG) {
        const int r = e / m, c = e % m;
        Lc[e] = (r < nb && c < nb) ? G[r * nb + c] + (r == c ? tau : 0.0) : 0.0;
        V[e] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int e = t; e < m * m; e += WG) {
            const double v = Lc[e];
            if (e / m == e % m) dia += v * v;
            else off += v * v;
        }
        off_s[t] = off;
        dia_s[t] = dia;
        __syncthreads();
        for (int h = WG / 2; h > 0; h >>= 1) {
            if (t < h) {
                off_s[t] += off_s[t + h];
                dia_s[t] += dia_s[t + h];
            }
            __syncthreads();
        }
        const double offt = off_s[0], diat = dia_s[0];
        __syncthreads();
        if (offt <= 1e-30 * diat || offt == 0.0) break;   // uniform
        for (int k = 0; k < m - 1; ++k) {
            // circle-method pairing: (m-1, k) and ((k+j) mod (m-1), (k-j) mod (m-1))
            if (t < m / 2) {
                int a1, b1;
                if (t == 0) {
                    a1 = m - 1;
                    b1 = k;
                } else {
                    a1 = (k + t) % (m - 1);
                    b1 = (k - t + (m - 1)) % (m - 1);
                }
                const int pp = min(a1, b1), qq = max(a1, b1);
                pp_s[t] = pp;
                pq_s[t] = qq;
                pair_of[pp] = t;
                side_of[pp] = 0;
                pair_of[qq] = t;
                side_of[qq] = 1;
                const double apq = Lc[pp * m + qq];
                double c = 1.0, sn = 0.0;
                if (apq != 0.0) {
                    const double tau = (Lc[qq * m + qq] - Lc[pp * m + pp]) / (2.0 * apq);
                    const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    sn = tt * c;
                }
                rc_s[t] = c;
                rs_s[t] = sn;
            }
            __syncthreads();
            // rows: Lc <- J^T Lc
            double nv[(MAXNB * MAXNB + WG - 1) / WG];
            for (int e = t, k2 = 0; e < m * m; e += WG, ++k2) {
                const int r = e / m, c2 = e % m, pr = pair_of[r];
                const double c = rc_s[pr], sn = rs_s[pr];
                const double vp = Lc[pp_s[pr] * m + c2], vq = Lc[pq_s[pr] * m + c2];
                nv[k2] = side_of[r] == 0 ? c * vp - sn * vq : sn * vp + c * vq;
            }
            __syncthreads();
            for (int e = t, k2 = 0; e < m * m; e += WG, ++k2) Lc[e] = nv[k2];
            __syncthreads();
            // columns: Lc <- Lc J, V <- V J
            double nw[(MAXNB * MAXNB + WG - 1) / WG];
            for (int e = t, k2 = 0; e < m * m; e += WG, ++k2) {
                const int r = e / m, c2 = e % m, pr = pair_of[c2];
                const double c = rc_s[pr], sn = rs_s[pr];
                const int p0 = pp_s[pr], q0 = pq_s[pr];
                const double lp = Lc[r * m + p0], lq = Lc[r * m + q0];
                const double vp = V[r * m + p0], vq = V[r * m + q0];
                nv[k2] = side_of[c2] == 0 ? c * lp - sn * lq : sn * lp + c * lq;
                nw[k2] = side_of[c2] == 0 ? c * vp - sn * vq : sn * vp + c * vq;
            }
            __syncthreads();
            for (int e = t, k2 = 0; e < m * m; e += WG, ++k2) {
                Lc[e] = nv[k2];
                V[e] = nw[k2];
            }
            __syncthreads();
        }
    }
    double emax = 0.0;
    for (int q = 0; q < nb; ++q) emax = fmax(emax, fabs(Lc[q * m + q]));
    // HV[r][a] = sum_u H[r][u] V[u][a] (into Aug)
    if (t < nb2) {
        const int r = t / nb, a2 = t % nb;
        double acc = 0.0;
        for (int u = 0; u < nb; ++u) acc += H[r * nb + u] * V[u * m + a2];
        Aug[t] = acc;
    }
    __syncthreads();
    if (t < nb2) {
        const int r = t / nb, c = t % nb;
        double acc = 0.0;
        for (int a2 = 0; a2 < nb; ++a2) {
            const double ev = Lc[a2 * m + a2];
            if (ev > PIVOT_TOL * emax) acc += Aug[r * nb + a2] * V[c * m + a2] / ev;
        }
        out[t] = acc;
    }
}

// Normal equations of one block row: G = M M^T, H = E M^T, Lambda~ = H G^{-1}
// (Cholesky; pseudo-inverse fallback).  A workgroup per list row, striding
// over the nl rows; with only != null over the only[0] list rows only[1..].
template <int NBT>   // > 0: block size fixed at compile time; 0: nb_rt
__global__ __launch_bounds__(WG) void k_gram_solve(int nl, const int32_t *__restrict__ list, int nb_rt,
                                                   const int32_t *__restrict__ mptr, const int32_t *__restrict__ mcol,
                                                   const double *__restrict__ mval, const int32_t *__restrict__ eptr,
                                                   const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                                   double *__restrict__ lamt, int32_t *__restrict__ singular,
                                                   double ridge, const int32_t *__restrict__ only) {
    __shared__ double G[MAXNB * MAXNB], H[MAXNB * MAXNB], Lc[MAXNB * MAXNB], V[MAXNB * MAXNB];
    __shared__ int32_t epos[UNION_CAP];   // position in pattern(M_i) of every block of E_i
  const int nrows = only ? only[0] : nl;
  for (int idx = blockIdx.x; idx < nrows; idx += gridDim.x) {
    const int li = only ? only[1 + idx] : idx;
    const int i = list[li];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int nb = NBT > 0 ? NBT : nb_rt;
    const int nb2 = nb * nb;
    const int mlo = mptr[li], k = mptr[li + 1] - mlo;
    const int elo = eptr[i], ek = eptr[i + 1] - elo;
    const bool epos_cached = ek <= UNION_CAP;
    if (epos_cached)
        for (int q = t; q < ek; q += WG) epos[q] = bsearch_i32(mcol, mlo, mlo + k, ecol[elo + q]);
    __syncthreads();
    // G = M M^T and H = E M^T as sums of column outer products: wavefront w owns
    // 4x4 tiles w, w+4, ... of G and H, its lanes split the columns, and the
    // tile sums are reduced across the lanes at the end.  Every lane reads
    // 4 + 4 entries of a column for 16 products of each matrix.
    const int ntd = (nb + 3) / 4;
    for (int tile = wave; tile < ntd * ntd; tile += WG / 64) {
        const int tr = (tile / ntd) * 4, tc = (tile % ntd) * 4;
        double ga[4][4], ha[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) ga[x][y] = ha[x][y] = 0.0;
#pragma unroll 2
        for (int j = lane; j < k * nb; j += 64) {
            const int pb = j / nb, u = j % nb;
            const double *mp = mval + (int64_t)(mlo + pb) * nb2 + u;
            double av[4], bv[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                av[x] = tr + x < nb ? mp[(tr + x) * nb] : 0.0;
                bv[x] = tc + x < nb ? mp[(tc + x) * nb] : 0.0;
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) ga[x][y] += av[x] * bv[y];
        }
#pragma unroll 2
        for (int j = lane; j < ek * nb; j += 64) {
            const int qb = j / nb, u = j % nb;
            const int pb = epos_cached ? epos[qb] : bsearch_i32(mcol, mlo, mlo + k, ecol[elo + qb]);
            if (pb < 0) continue;   // pattern(E_i) is contained in pattern(M_i)
            const double *ep = eval + (int64_t)(elo + qb) * nb2 + u;
            const double *mp = mval + (int64_t)pb * nb2 + u;
            double av[4], bv[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                av[x] = tr + x < nb ? ep[(tr + x) * nb] : 0.0;
                bv[x] = tc + x < nb ? mp[(tc + x) * nb] : 0.0;
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) ha[x][y] += av[x] * bv[y];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    ga[x][y] += __shfl_xor(ga[x][y], off, 64);
                    ha[x][y] += __shfl_xor(ha[x][y], off, 64);
                }
        }
        if (lane == 0) {
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y)
                    if (tr + x < nb && tc + y < nb) {
                        G[(tr + x) * nb + tc + y] = ga[x][y];
                        H[(tr + x) * nb + tc + y] = ha[x][y];
                    }
        }
    }
    __syncthreads();
    normal_solve(G, H, Lc, V, nb, lamt + (int64_t)i * nb2, singular + li, ridge);
    __syncthreads();   // G, H and epos are rewritten by the next row
  }
}

// G = M M^T and H = E M^T on the matrix cores (FP64 MFMA 16x16x4) for 16x16
// blocks.  Operand lanes: A lane l = A[l%16][l/16], B lane l = B[l/16][l%16],
// result lane l, register i = D[4i + l/16][l%16].  With B = the next four
// columns of M (transposed), a lane's B value is its own A value of M; two
// chains, A = M (G) and A = E (H).  Wavefront w sums the blocks p = w, w + 4,
// ... of the row; the four partial sums are added in LDS in wave order, then
// the normal equations are solved as in k_gram_solve.  (For 8x8 blocks the
// VALU kernel measured faster: half of every 16x16 product would be idle.)
typedef double d4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(WG) void k_gram_mfma(const int32_t *__restrict__ list,
                                                  const int32_t *__restrict__ mptr, const int32_t *__restrict__ mcol,
                                                  const double *__restrict__ mval, const int32_t *__restrict__ eptr,
                                                  const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                                  double *__restrict__ lamt, int32_t *__restrict__ singular,
                                                  double ridge) {
    constexpr int NBT = 16, NB2 = NBT * NBT, QCAP = 4096;
    __shared__ double G[MAXNB * MAXNB], H[MAXNB * MAXNB], Lc[MAXNB * MAXNB], V[MAXNB * MAXNB];
    __shared__ double part[WG / 64][2][16][16];
    __shared__ int32_t qpos[QCAP];   // position in E_i of every block of M_i (-1: none)
    const int li = blockIdx.x;
    const int i = list[li];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int mlo = mptr[li], k = mptr[li + 1] - mlo;
    const int elo = eptr[i], ek = eptr[i + 1] - elo;
    const bool cached = k <= QCAP;
    if (cached)
        for (int p = t; p < k; p += WG) qpos[p] = bsearch_i32(ecol, elo, elo + ek, mcol[mlo + p]);
    __syncthreads();
    const int r = lane & 15, cq = lane >> 4;   // operand row, column within the group of four
    d4_t dg = {0.0, 0.0, 0.0, 0.0}, dh = {0.0, 0.0, 0.0, 0.0};
    for (int p = wave; p < k; p += WG / 64) {
        const int q = cached ? qpos[p] : bsearch_i32(ecol, elo, elo + ek, mcol[mlo + p]);
        const double *mb = mval + (int64_t)(mlo + p) * NB2;
        const double *eb = eval + (int64_t)(q >= 0 ? q : 0) * NB2;   // block 0 when q < 0: read, then discarded
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * j + cq;
            const double am = mb[r * 16 + c];
            const double ve = eb[r * 16 + c];   // eb is a valid block even when q < 0
            const double ae = q >= 0 ? ve : 0.0;
            dg = __builtin_amdgcn_mfma_f64_16x16x4f64(am, am, dg, 0, 0, 0);
            dh = __builtin_amdgcn_mfma_f64_16x16x4f64(ae, am, dh, 0, 0, 0);
        }
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        part[wave][0][4 * x + cq][r] = dg[x];
        part[wave][1][4 * x + cq][r] = dh[x];
    }
    __syncthreads();
    for (int e = t; e < NB2; e += WG) {
        const int x = e / NBT, y = e % NBT;
        double g = 0.0, h = 0.0;
#pragma unroll
        for (int w = 0; w < WG / 64; ++w) {
            g += part[w][0][x][y];
            h += part[w][1][x][y];
        }
        G[e] = g;
        H[e] = h;
    }
    __syncthreads();
    normal_solve(G, H, Lc, V, NBT, lamt + (int64_t)i * NB2, singular + li, ridge);
}

// G = M M^T and H = E M^T for 8x8 blocks on the FP64 matrix cores, two block
// rows per wavefront: operand rows 0-7 of a 16x16x4 product belong to the
// first row, rows 8-15 to the second, so the two diagonal 8x8 blocks of the
// 16x16 result are the two rows' Gram matrices (the off-diagonal blocks pair
// columns of different rows and are discarded).  A step takes four columns of
// each row's M, two steps per block; the shorter row is padded with zeros.
// The position in E_i of every block of M_i is searched first, by the whole
// workgroup, into LDS (rows of more than QCAP8 blocks search as they go), so
// that the product loop's iterations are independent.  The normal equations
// of the workgroup's eight rows are then solved together with normal_solve's
// Gauss-Jordan elimination, pivot cut-off and product order; a row that meets
// a pivot below the cut-off (or a non-positive diagonal) gets redo[li] = 1
// and is appended to redo_list (count in redo_list[0], rows from index 1) for
// k_gram_solve's minimum-norm path.
constexpr int QCAP8 = 256;
constexpr int ECAP8 = 128;   // E_i column lists staged per row in k_gram_mfma8

__global__ __launch_bounds__(WG, 8) void k_gram_mfma8(int nl, const int32_t *__restrict__ list,
                                                   const int32_t *__restrict__ mptr, const int32_t *__restrict__ mcol,
                                                   const double *__restrict__ mval, const int32_t *__restrict__ eptr,
                                                   const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                                   double *__restrict__ lamt, int32_t *__restrict__ redo,
                                                   int32_t *__restrict__ redo_list, double ridge) {
    constexpr int NB = 8, NB2 = 64, W2 = 2 * NB, ROWS = 2 * (WG / 64);
    // one LDS buffer for the two phases: the positions and E_i's column lists
    // while the products run, then G, H and [G + tau I | I] (16 KB instead of
    // 28 KB: more workgroups per CU)
    constexpr size_t P1 = sizeof(int32_t) * ROWS * (QCAP8 + ECAP8);
    constexpr size_t P2 = sizeof(double) * ROWS * (2 * NB2 + NB * W2);
    __shared__ __align__(16) unsigned char lds[P1 > P2 ? P1 : P2];
    int32_t(*qpos)[QCAP8] = reinterpret_cast<int32_t(*)[QCAP8]>(lds);
    int32_t(*ecs8)[ECAP8] = reinterpret_cast<int32_t(*)[ECAP8]>(lds + sizeof(int32_t) * ROWS * QCAP8);
    double(*Gs)[NB2] = reinterpret_cast<double(*)[NB2]>(lds);
    double(*Hs)[NB2] = Gs + ROWS;
    double(*Aug)[NB * W2] = reinterpret_cast<double(*)[NB * W2]>(lds + sizeof(double) * ROWS * 2 * NB2);
    __shared__ int32_t rmlo[ROWS], rk[ROWS], relo[ROWS], rek[ROWS];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int r16 = lane & 15, cq = lane >> 4, half = r16 >> 3, rr = r16 & 7;
    const int slot = 2 * wave + half;
    if (t < ROWS) {
        const int lr = blockIdx.x * ROWS + t;
        int a = 0, b = 0, c = 0, d = 0;
        if (lr < nl) {
            const int i = list[lr];
            a = mptr[lr];
            b = mptr[lr + 1] - a;
            c = eptr[i];
            d = eptr[i + 1] - c;
        }
        rmlo[t] = a;
        rk[t] = b;
        relo[t] = c;
        rek[t] = d;
    }
    __syncthreads();
    // The positions of M_i's block columns in E_i, for the eight rows at once:
    // E_i's column lists are staged in LDS with coalesced reads, so the
    // searches run in LDS instead of as chains of dependent global loads.
    __shared__ int32_t qoff[ROWS + 1];
    for (int e = t; e < ROWS * ECAP8; e += WG) {
        const int sr = e / ECAP8, q = e % ECAP8;
        if (q < rek[sr] && rek[sr] <= ECAP8) ecs8[sr][q] = ecol[relo[sr] + q];
    }
    if (t == 0) {
        qoff[0] = 0;
        for (int sr = 0; sr < ROWS; ++sr) qoff[sr + 1] = qoff[sr] + min(rk[sr], QCAP8);
    }
    __syncthreads();
    for (int e = t; e < qoff[ROWS]; e += WG) {
        int sr = 0;
        while (qoff[sr + 1] <= e) ++sr;
        const int p = e - qoff[sr];
        const int key = mcol[rmlo[sr] + p];
        int q;
        if (rek[sr] <= ECAP8) {
            q = bsearch_i32(ecs8[sr], 0, rek[sr], key);
            if (q >= 0) q += relo[sr];
        } else {
            q = bsearch_i32(ecol, relo[sr], relo[sr] + rek[sr], key);
        }
        qpos[sr][p] = q;
    }
    __syncthreads();
    const int mlo = rmlo[slot], k = rk[slot], elo = relo[slot], ek = rek[slot];
    const int kmax = max(rk[2 * wave], rk[2 * wave + 1]);   // wave-uniform trip count
    d4_t dg = {0.0, 0.0, 0.0, 0.0}, dh = {0.0, 0.0, 0.0, 0.0};
    // PB block columns per pass: their M and E loads are all issued before the
    // first product (one memory round trip per pass instead of per column); the
    // products run in column order as one at a time would.  Two columns, with
    // the accumulators in ordinary registers (56 VGPRs) and the two-phase LDS
    // (16.5 KB), run eight waves per SIMD; on the 128^3 setup that measured
    // faster than four columns at five waves (51.1 -> 50.1 ms) and eight at four
    constexpr int PB = 2;
    for (int p0 = 0; p0 < kmax; p0 += PB) {
        double am0[PB], am1[PB], ae0[PB], ae1[PB];
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            const int p = p0 + u;
            am0[u] = am1[u] = ae0[u] = ae1[u] = 0.0;
            if (p < k) {
                const int q = p < QCAP8 ? qpos[slot][p] : bsearch_i32(ecol, elo, elo + ek, mcol[mlo + p]);
                const double *mb = mval + (int64_t)(mlo + p) * NB2 + rr * NB;
                am0[u] = mb[cq];
                am1[u] = mb[4 + cq];
                if (q >= 0) {
                    const double *eb = eval + (int64_t)q * NB2 + rr * NB;
                    ae0[u] = eb[cq];
                    ae1[u] = eb[4 + cq];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            if (p0 + u >= kmax) break;   // wave-uniform
            dg = __builtin_amdgcn_mfma_f64_16x16x4f64(am0[u], am0[u], dg, 0, 0, 0);
            dh = __builtin_amdgcn_mfma_f64_16x16x4f64(ae0[u], am0[u], dh, 0, 0, 0);
            dg = __builtin_amdgcn_mfma_f64_16x16x4f64(am1[u], am1[u], dg, 0, 0, 0);
            dh = __builtin_amdgcn_mfma_f64_16x16x4f64(ae1[u], am1[u], dh, 0, 0, 0);
        }
    }
    __syncthreads();   // every wave is done with the positions (phase 1 of lds)
    // result lane l, register x = D[4x + l/16][l%16]: this lane's half owns
    // registers 2 half and 2 half + 1 of its own column
    {
        const double g0 = half ? dg[2] : dg[0], g1 = half ? dg[3] : dg[1];
        const double h0 = half ? dh[2] : dh[0], h1 = half ? dh[3] : dh[1];
        Gs[slot][cq * NB + rr] = g0;
        Gs[slot][(4 + cq) * NB + rr] = g1;
        Hs[slot][cq * NB + rr] = h0;
        Hs[slot][(4 + cq) * NB + rr] = h1;
    }
    __syncthreads();
    // eight rows, 32 threads each, four entries of [G + tau I | I] per thread
    const int s = t >> 5, j = t & 31;
    const int ls = blockIdx.x * ROWS + s;
    const double *G = Gs[s];
    double trace = 0.0, dmax = 0.0;
    for (int q = 0; q < NB; ++q) trace += G[q * NB + q];
    const double tau = ridge > 0.0 ? ridge * trace / NB : 0.0;
    for (int q = 0; q < NB; ++q) dmax = fmax(dmax, G[q * NB + q] + tau);
    bool bad = !(dmax > 0.0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int e = j + 32 * m, r = e / W2, c = e % W2;
        Aug[s][e] = c < NB ? G[r * NB + c] + (r == c ? tau : 0.0) : (c - NB == r ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int q = 0; q < NB; ++q) {   // uniform: every slot takes all NB steps, a bad one without updates
        const double piv = Aug[s][q * W2 + q];
        if (!(piv > PIVOT_TOL * dmax)) bad = true;
        double f[4], g[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int e = j + 32 * m;
            f[m] = Aug[s][(e / W2) * W2 + q];
            g[m] = Aug[s][q * W2 + e % W2];
        }
        __syncthreads();
        if (!bad) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int e = j + 32 * m;
                Aug[s][e] = (e / W2 == q) ? g[m] / piv : Aug[s][e] - f[m] * g[m] / piv;
            }
        }
        __syncthreads();
    }
    if (ls >= nl) return;
    if (j == 0) {
        redo[ls] = bad ? 1 : 0;
        if (bad) redo_list[1 + atomicAdd(redo_list, 1)] = ls;
    }
    if (bad) return;
    const int i = list[ls];
    const double *H = Hs[s];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int e = j + 32 * m, r = e / NB, c = e % NB;
        double acc = 0.0;
        for (int u = 0; u < NB; ++u) acc += H[r * NB + u] * Aug[s][u * W2 + NB + c];
        lamt[(int64_t)i * NB2 + e] = acc;
    }
}

// Point blocks (n = 1): one wavefront per list row, four rows per workgroup.
// M_i[p] = sum_j a~_ij E_j[col p]; Lambda~_i = H_i / G_i with G_i = sum M_i^2,
// H_i = sum E_i M_i (0 when G_i = 0, the minimum-norm solution).  Lane striding
// and the reduction order are those of the blocked kernels.
__global__ __launch_bounds__(WG) void k_rowprod_point(int nl, const int32_t *__restrict__ list,
                                                      const int32_t *__restrict__ abptr,
                                                      const int32_t *__restrict__ abcol,
                                                      const double *__restrict__ abval,
                                                      const int32_t *__restrict__ eptr,
                                                      const int32_t *__restrict__ ecol,
                                                      const double *__restrict__ eval,
                                                      const int32_t *__restrict__ mptr,
                                                      const int32_t *__restrict__ mcol, double *__restrict__ mval) {
    // see k_rowprod_nb for the order of the rows
    const int w = (int)xcd_tile(blockIdx.x, gridDim.x) * (WG / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (w >= nl) return;
    const int i = list[w];
    const int alo = abptr[i], deg = abptr[i + 1] - alo;
    const int mlo = mptr[w], k = mptr[w + 1] - mlo;
    for (int p = lane; p < k; p += 64) {
        const int col = mcol[mlo + p];
        double acc = 0.0;
        for (int jj = 0; jj < deg; ++jj) {
            const int j = abcol[alo + jj];
            const int q = bsearch_i32(ecol, eptr[j], eptr[j + 1], col);
            if (q >= 0) acc += abval[alo + jj] * eval[q];
        }
        mval[mlo + p] = acc;
    }
}

__global__ __launch_bounds__(WG) void k_gram_point(int nl, const int32_t *__restrict__ list,
                                                   const int32_t *__restrict__ mptr, const int32_t *__restrict__ mcol,
                                                   const double *__restrict__ mval, const int32_t *__restrict__ eptr,
                                                   const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                                   double *__restrict__ lamt, int32_t *__restrict__ singular,
                                                   double ridge) {
    const int w = blockIdx.x * (WG / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (w >= nl) return;
    const int i = list[w];
    const int mlo = mptr[w], k = mptr[w + 1] - mlo;
    const int elo = eptr[i], ek = eptr[i + 1] - elo;
    double g = 0.0, h = 0.0;
    for (int p = lane; p < k; p += 64) g += mval[mlo + p] * mval[mlo + p];
    for (int q = lane; q < ek; q += 64) {
        const int pb = bsearch_i32(mcol, mlo, mlo + k, ecol[elo + q]);
        if (pb >= 0) h += eval[elo + q] * mval[pb];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        g += __shfl_xor(g, off, 64);
        h += __shfl_xor(h, off, 64);
    }
    if (lane == 0) {
        const bool bad = !(g > 0.0);
        singular[w] = bad ? 1 : 0;
        lamt[i] = bad ? 0.0 : h / (g + (ridge > 0.0 ? ridge * g : 0.0));   // tr(G_i) / 1 = g
    }
}

// ---------------------------------------------------------------------------
// sketched construction (Sec. 4): the residual E_{l-1} is replaced by the
// N x s sketch T = E_{l-1} S (row-major, s <= 64).  One wavefront per list
// block, lane c = sketch column c; the rows of A are read through the scalar
// CSR (uniform per wavefront) and T rows are gathered whole (coalesced).
// ---------------------------------------------------------------------------
constexpr int SK_MAX = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// m[r] = (A~ T)[i n + r][c], t[r] = T[i n + r][c] with A~ = W A W
template <int NB>
__device__ __forceinline__ void sk_rows(int i, int lane, int s, const int32_t *__restrict__ aptr,
                                        const int32_t *__restrict__ acol, const double *__restrict__ aval,
                                        const double *__restrict__ w, const double *__restrict__ T,
                                        double (&m)[NB], double (&t)[NB]) {
    const bool on = lane < s;
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        const int64_t row = (int64_t)i * NB + r;
        double acc = 0.0;
        for (int e = aptr[row]; e < aptr[row + 1]; ++e) {
            const int k = acol[e];
            const double tk = on ? T[(int64_t)k * s + lane] : 0.0;
            acc += aval[e] * w[k] * tk;
        }
        m[r] = w[row] * acc;
        t[r] = on ? T[row * s + lane] : 0.0;
    }
}

// Point blocks: Lambda~_i = (T_i, M_i) / (M_i, M_i) (0 when M_i = 0, the
// minimum-norm solution) and T_i <- T_i - Lambda~_i M_i, written to Tout.
__global__ __launch_bounds__(WG) void k_sk_point(int nl, const int32_t *__restrict__ list,
                                                 const int32_t *__restrict__ aptr, const int32_t *__restrict__ acol,
                                                 const double *__restrict__ aval, const double *__restrict__ w, int s,
                                                 const double *T, double *Tout, double *__restrict__ lamt,
                                                 int32_t *__restrict__ singular) {
    const int wi = blockIdx.x * (WG / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (wi >= nl) return;   // whole wavefront
    const int i = list[wi];
    double m[1], t[1];
    sk_rows<1>(i, lane, s, aptr, acol, aval, w, T, m, t);
    const double g = wave_sum(m[0] * m[0]), h = wave_sum(t[0] * m[0]);
    const bool bad = !(g > 0.0);
    const double lam = bad ? 0.0 : h / g;
    if (lane == 0) {
        lamt[i] = lam;
        singular[wi] = bad ? 1 : 0;
    }
    if (lane < s) Tout[(int64_t)i * s + lane] = t[0] - lam * m[0];
}

// Block rows: M_i to Mb[wi][NB][s], G_i = M_i M_i^T and H_i = T_i M_i^T to
// gh[wi][2][NB][NB]
template <int NB>
__global__ __launch_bounds__(WG) void k_sk_gram(int nl, const int32_t *__restrict__ list,
                                                const int32_t *__restrict__ aptr, const int32_t *__restrict__ acol,
                                                const double *__restrict__ aval, const double *__restrict__ w, int s,
                                                const double *__restrict__ T, double *__restrict__ Mb,
                                                double *__restrict__ gh) {
    const int wi = blockIdx.x * (WG / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (wi >= nl) return;
    const int i = list[wi];
    double m[NB], t[NB];
    sk_rows<NB>(i, lane, s, aptr, acol, aval, w, T, m, t);
    if (lane < s) {
#pragma unroll
        for (int r = 0; r < NB; ++r) Mb[((int64_t)wi * NB + r) * s + lane] = m[r];
    }
    double *g = gh + (int64_t)wi * 2 * NB * NB, *h = g + NB * NB;
#pragma unroll
    for (int p = 0; p < NB; ++p) {
#pragma unroll
        for (int q = 0; q <= p; ++q) {
            const double v = wave_sum(m[p] * m[q]);
            if (lane == 0) {
                g[p * NB + q] = v;
                g[q * NB + p] = v;
            }
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const double v = wave_sum(t[p] * m[q]);
            if (lane == 0) h[p * NB + q] = v;
        }
    }
}

// Lambda~_i G_i = H_i per list block (the exact fit's solve), one workgroup each
__global__ __launch_bounds__(WG) void k_sk_solve(const int32_t *__restrict__ list, int nb,
                                                 const double *__restrict__ gh, double *__restrict__ lamt,
                                                 int32_t *__restrict__ singular, double ridge) {
    __shared__ double G[MAXNB * MAXNB], H[MAXNB * MAXNB], Lc[MAXNB * MAXNB], V[MAXNB * MAXNB];
    const int wi = blockIdx.x, nb2 = nb * nb;
    const double *src = gh + (int64_t)wi * 2 * nb2;
    for (int e = threadIdx.x; e < nb2; e += WG) {
        G[e] = src[e];
        H[e] = src[nb2 + e];
    }
    __syncthreads();
    normal_solve(G, H, Lc, V, nb, lamt + (int64_t)list[wi] * nb2, singular + wi, ridge);
}

// ---- overlapping blocks (Sec. 3.6.2), sketched form -------------------------
// M = A~ T on every row (one wavefront per row, lane = sketch column)
__global__ __launch_bounds__(WG) void k_sk_rows(int64_t n, const int32_t *__restrict__ aptr,
                                                const int32_t *__restrict__ acol, const double *__restrict__ aval,
                                                const double *__restrict__ w, int s, const double *__restrict__ T,
                                                double *__restrict__ M) {
    const int64_t row = blockIdx.x * (int64_t)(WG / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n || lane >= s) return;
    double acc = 0.0;
    for (int e = aptr[row]; e < aptr[row + 1]; ++e) {
        const int k = acol[e];
        acc += aval[e] * w[k] * T[(int64_t)k * s + lane];
    }
    M[row * s + lane] = w[row] * acc;
}

// G_i = M_i M_i^T, H_i = T_i M_i^T over the block's slots (unused slots: zero
// rows) into gh[i][2][m][m]
template <int MB>
__global__ __launch_bounds__(WG) void k_ovl_gram(int64_t nblk, int m, const int32_t *__restrict__ nodes, int s,
                                                 const double *__restrict__ M, const double *__restrict__ T,
                                                 double *__restrict__ gh) {
    const int64_t wi = blockIdx.x * (int64_t)(WG / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wi >= nblk) return;
    double mv[MB], tv[MB];
#pragma unroll
    for (int r = 0; r < MB; ++r) {
        const int k = r < m ? nodes[wi * m + r] : -1;
        mv[r] = (k >= 0 && lane < s) ? M[(int64_t)k * s + lane] : 0.0;
        tv[r] = (k >= 0 && lane < s) ? T[(int64_t)k * s + lane] : 0.0;
    }
    double *g = gh + wi * 2 * m * m, *h = g + m * m;
#pragma unroll
    for (int p = 0; p < MB; ++p) {
        if (p >= m) break;   // uniform
#pragma unroll
        for (int q = 0; q < MB; ++q) {
            if (q >= m) break;
            const double gv = q <= p ? wave_sum(mv[p] * mv[q]) : 0.0;
            const double hv = wave_sum(tv[p] * mv[q]);
            if (lane == 0) {
                if (q <= p) {
                    g[p * m + q] = gv;
                    g[q * m + p] = gv;
                }
                h[p * m + q] = hv;
            }
        }
    }
}

// Y[i][r][c] = sum_u Lambda~_i[r][u] M[node(i, u)][c]
template <int MB>
__global__ __launch_bounds__(WG) void k_ovl_y(int64_t nblk, int m, const int32_t *__restrict__ nodes, int s,
                                              const double *__restrict__ lamt, const double *__restrict__ M,
                                              double *__restrict__ Y) {
    const int64_t wi = blockIdx.x * (int64_t)(WG / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wi >= nblk || lane >= s) return;
    double mv[MB];
#pragma unroll
    for (int u = 0; u < MB; ++u) {
        const int k = u < m ? nodes[wi * m + u] : -1;
        mv[u] = k >= 0 ? M[(int64_t)k * s + lane] : 0.0;
    }
    const double *lam = lamt + wi * m * m;
    for (int r = 0; r < m; ++r) {
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < MB; ++u)
            if (u < m) v += lam[r * m + u] * mv[u];
        Y[(wi * m + r) * s + lane] = v;
    }
}

// T[k][c] <- T[k][c] - (1 / theta_k) sum over the slots of k of Y[slot][c]
__global__ __launch_bounds__(WG) void k_ovl_fuse_T(int64_t n, const int32_t *__restrict__ iptr,
                                                   const int32_t *__restrict__ iidx,
                                                   const double *__restrict__ rtheta, int s,
                                                   const double *__restrict__ Y, double *__restrict__ T) {
    const int64_t k = blockIdx.x * (int64_t)(WG / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= n || lane >= s) return;
    double acc = 0.0;
    for (int q = iptr[k]; q < iptr[k + 1]; ++q) acc += Y[(int64_t)iidx[q] * s + lane];
    T[k * s + lane] -= rtheta[k] * acc;
}

// Lambda_i = W_i Lambda~_i W_i over the block's nodes (unused slots: zero)
__global__ void k_ovl_unscale(int64_t nblk, int m, const int32_t *__restrict__ nodes, const double *__restrict__ w,
                              const double *__restrict__ lamt, double *__restrict__ lam) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= nblk * m * m) return;
    const int64_t i = e / (m * m);
    const int r = (int)(e / m % m), c = (int)(e % m);
    const int kr = nodes[i * m + r], kc = nodes[i * m + c];
    lam[e] = (kr >= 0 && kc >= 0) ? w[kr] * lamt[e] * w[kc] : 0.0;
}

// ---- overlapping blocks, exact form (Sec. 3.6.2): scalar residual E ----------
// Prescaled values of A on its own pattern: a~_jl = w_j a_jl w_l
__global__ void k_prescaled_csr(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                const double *__restrict__ val, const double *__restrict__ w,
                                double *__restrict__ out) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int k = ptr[r]; k < ptr[r + 1]; ++k) out[k] = w[r] * val[k] * w[col[k]];
}

// value of row (ptr, col, val) at column c, 0 when absent
__device__ __forceinline__ double row_at(const int32_t *col, const double *val, int lo, int hi, int32_t c) {
    const int q = bsearch_i32(col, lo, hi, c);
    return q >= 0 ? val[q] : 0.0;
}

// G_i[s][t] = M_{n(s)} . M_{n(t)},  H_i[s][t] = E_{n(s)} . M_{n(t)} (sparse rows,
// unused slots zero), one wavefront per block; gh[i][2][m][m]
__global__ __launch_bounds__(WG) void k_ovl_gram_sparse(int64_t nblk, int m, const int32_t *__restrict__ nodes,
                                                        const int32_t *__restrict__ mptr,
                                                        const int32_t *__restrict__ mcol,
                                                        const double *__restrict__ mval,
                                                        const int32_t *__restrict__ eptr,
                                                        const int32_t *__restrict__ ecol,
                                                        const double *__restrict__ eval, double *__restrict__ gh) {
    const int64_t wi = blockIdx.x * (int64_t)(WG / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wi >= nblk) return;
    double *g = gh + wi * 2 * m * m, *h = g + m * m;
    for (int sI = 0; sI < m; ++sI) {
        const int a = nodes[wi * m + sI];
        for (int tI = 0; tI < m; ++tI) {
            const int bn = nodes[wi * m + tI];
            double gv = 0.0, hv = 0.0;
            if (a >= 0 && bn >= 0) {
                const int b0 = mptr[bn], b1 = mptr[bn + 1];
                if (tI >= sI)
                    for (int q = mptr[a] + lane; q < mptr[a + 1]; q += 64)
                        gv += mval[q] * row_at(mcol, mval, b0, b1, mcol[q]);
                for (int q = eptr[a] + lane; q < eptr[a + 1]; q += 64)
                    hv += eval[q] * row_at(mcol, mval, b0, b1, ecol[q]);
            }
            gv = wave_sum(gv);
            hv = wave_sum(hv);
            if (lane == 0) {
                if (tI >= sI) {
                    g[sI * m + tI] = gv;
                    g[tI * m + sI] = gv;
                }
                h[sI * m + tI] = hv;
            }
        }
    }
}

// Rows that feed node k's new residual row: E_k itself, then the M rows of
// every node u of every block holding k.  Returns the number of segments;
// seg_row[s] < 0 marks the E row.
__device__ __forceinline__ int ovl_segments(int k, int m, const int32_t *__restrict__ nodes,
                                            const int32_t *__restrict__ iptr, const int32_t *__restrict__ iidx,
                                            int32_t *seg_row, int cap) {
    int ns = 0;
    seg_row[ns++] = -1;
    for (int q = iptr[k]; q < iptr[k + 1]; ++q) {
        const int i = iidx[q] / m;
        for (int u = 0; u < m; ++u) {
            const int node = nodes[(int64_t)i * m + u];
            if (node >= 0 && ns < cap) seg_row[ns++] = node;
        }
    }
    return ns;
}

// Symbolic new residual row of node k: the sorted union of the columns of its
// segments (one workgroup per node, bitonic sort in LDS as k_union).
template <bool FILL>
__global__ __launch_bounds__(WG) void k_ovl_union(int64_t n, int m, const int32_t *__restrict__ nodes,
                                                  const int32_t *__restrict__ iptr, const int32_t *__restrict__ iidx,
                                                  const int32_t *__restrict__ eptr, const int32_t *__restrict__ ecol,
                                                  const int32_t *__restrict__ mptr, const int32_t *__restrict__ mcol,
                                                  int32_t *__restrict__ out_cnt, const int32_t *__restrict__ out_ptr,
                                                  int32_t *__restrict__ out_col, int32_t *__restrict__ err) {
    __shared__ int32_t cand[UNION_CAP_BIG];
    __shared__ int32_t seg_row[256], offs[257];
    __shared__ int32_t part[WG + 1];
    __shared__ int nseg_s;
    const int64_t k = blockIdx.x;
    const int t = threadIdx.x;
    if (t == 0) {
        nseg_s = ovl_segments((int)k, m, nodes, iptr, iidx, seg_row, 256);
        offs[0] = 0;
        for (int q = 0; q < nseg_s; ++q) {
            const int r = seg_row[q];
            offs[q + 1] = offs[q] + (r < 0 ? eptr[k + 1] - eptr[k] : mptr[r + 1] - mptr[r]);
        }
    }
    __syncthreads();
    const int nseg = nseg_s, total = offs[nseg];
    if (total > UNION_CAP_BIG) {
        if (t == 0) {
            err[k] = 1;
            if (!FILL) out_cnt[k] = 0;
        }
        return;
    }
    for (int e = t; e < total; e += WG) {
        int q = 0;
        while (offs[q + 1] <= e) ++q;
        const int r = seg_row[q];
        cand[e] = r < 0 ? ecol[eptr[k] + (e - offs[q])] : mcol[mptr[r] + (e - offs[q])];
    }
    int P = 1;
    while (P < total) P <<= 1;
    for (int e = total + t; e < P; e += WG) cand[e] = INT32_MAX;
    __syncthreads();
    for (int kk = 2; kk <= P; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int a = t; a < P; a += WG) {
                const int b = a ^ j;
                if (b > a) {
                    const int32_t x = cand[a], y = cand[b];
                    const bool up = (a & kk) == 0;
                    if ((x > y) == up) {
                        cand[a] = y;
                        cand[b] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    const int chunk = (P + WG - 1) / WG;
    const int a0 = t * chunk, a1 = min(P, a0 + chunk);
    int mine = 0;
    for (int a = a0; a < a1; ++a) {
        const int32_t v = cand[a];
        if (v != INT32_MAX && (a == 0 || cand[a - 1] != v)) ++mine;
    }
    part[t + 1] = mine;
    __syncthreads();
    if (t == 0) {
        part[0] = 0;
        for (int q = 0; q < WG; ++q) part[q + 1] += part[q];
    }
    __syncthreads();
    if (!FILL) {
        if (t == 0) out_cnt[k] = part[WG];
    } else {
        int o = out_ptr[k] + part[t];
        for (int a = a0; a < a1; ++a) {
            const int32_t v = cand[a];
            if (v != INT32_MAX && (a == 0 || cand[a - 1] != v)) out_col[o++] = v;
        }
    }
}

// Numeric new residual row of node k on its pattern:
//   E_new[k][c] = E[k][c] - (1/theta_k) sum_{(i,s) holding k} sum_u Lambda~_i[s][u] M[n(i,u)][c]
// one wavefront per node, each lane owns output positions (fixed summation order)
__global__ __launch_bounds__(WG) void k_ovl_eupdate(int64_t n, int m, const int32_t *__restrict__ nodes,
                                                    const int32_t *__restrict__ iptr,
                                                    const int32_t *__restrict__ iidx,
                                                    const double *__restrict__ rtheta,
                                                    const double *__restrict__ lamt, const int32_t *__restrict__ eptr,
                                                    const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                                    const int32_t *__restrict__ mptr, const int32_t *__restrict__ mcol,
                                                    const double *__restrict__ mval, const int32_t *__restrict__ nptr,
                                                    const int32_t *__restrict__ ncol, double *__restrict__ nval) {
    const int64_t k = blockIdx.x * (int64_t)(WG / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= n) return;
    const double rt = rtheta[k];
    for (int p = nptr[k] + lane; p < nptr[k + 1]; p += 64) {
        const int32_t c = ncol[p];
        double v = row_at(ecol, eval, eptr[k], eptr[k + 1], c);
        for (int q = iptr[k]; q < iptr[k + 1]; ++q) {
            const int64_t i = iidx[q] / m;
            const int sl = iidx[q] % m;
            const double *lam = lamt + (i * m + sl) * m;
            for (int u = 0; u < m; ++u) {
                const int node = nodes[i * m + u];
                if (node < 0) continue;
                v -= rt * lam[u] * row_at(mcol, mval, mptr[node], mptr[node + 1], c);
            }
        }
        nval[p] = v;
    }
}

// T_i <- T_i - Lambda~_i M_i for the list blocks (in place: M was formed from
// the old T before this launch)
template <int NB>
__global__ __launch_bounds__(WG) void k_sk_update(int nl, const int32_t *__restrict__ list, int s,
                                                  const double *__restrict__ lamt, const double *__restrict__ Mb,
                                                  double *__restrict__ T) {
    const int wi = blockIdx.x * (WG / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (wi >= nl || lane >= s) return;
    const int i = list[wi];
    const double *lam = lamt + (int64_t)i * NB * NB;
    double m[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) m[u] = Mb[((int64_t)wi * NB + u) * s + lane];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        double v = T[((int64_t)i * NB + r) * s + lane];
#pragma unroll
        for (int u = 0; u < NB; ++u) v -= lam[r * NB + u] * m[u];
        T[((int64_t)i * NB + r) * s + lane] = v;
    }
}

// E_new,i = E_old,i - Lambda~_i M_i for list rows (on pattern(M_i)); other rows
// are copied.  One workgroup per block row.
// NBT > 0: block size fixed at compile time (Lambda row in registers, the M
// column loads unrolled); NBT = 0: nb at run time.
template <int NBT>
__global__ __launch_bounds__(WG) void k_eupdate(int B, int nb_rt, const int32_t *__restrict__ pos_in_list,
                                                const int32_t *__restrict__ mptr, const int32_t *__restrict__ mcol,
                                                const double *__restrict__ mval, const int32_t *__restrict__ eptr,
                                                const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                                const double *__restrict__ lamt, const int32_t *__restrict__ nptr,
                                                int32_t *__restrict__ ncol, double *__restrict__ nval) {
    constexpr int QCAP = NBT == 1 ? 256 : 4096;   // block positions of a row kept in LDS (point rows are short)
    __shared__ int32_t qpos[QCAP];
    const int i = blockIdx.x;
    if (i >= B) return;
    const int t = threadIdx.x;
    const int nb = NBT > 0 ? NBT : nb_rt;
    const int nb2 = nb * nb;
    const int li = pos_in_list[i];
    if (li == -2) return;   // member of a lattice class: translated from its representative
    const int elo = eptr[i], ek = eptr[i + 1] - elo;
    const int nlo = nptr[i];
    if (li < 0) {   // unchanged row: copy (16-byte accesses, four in flight per thread)
        for (int q = t; q < ek; q += WG) ncol[nlo + q] = ecol[elo + q];
        const int64_t n = (int64_t)ek * nb2;
        const double *src = eval + (int64_t)elo * nb2;
        double *dst = nval + (int64_t)nlo * nb2;
        if ((nb2 & 1) == 0) {   // row starts are then 16-byte aligned
            const double2 *s2 = reinterpret_cast<const double2 *>(src);
            double2 *d2 = reinterpret_cast<double2 *>(dst);
            const int64_t n2 = n / 2;
            int64_t e = t;
            for (; e + 3 * WG < n2; e += 4 * WG) {
                const double2 a0 = s2[e], a1 = s2[e + WG], a2 = s2[e + 2 * WG], a3 = s2[e + 3 * WG];
                d2[e] = a0;
                d2[e + WG] = a1;
                d2[e + 2 * WG] = a2;
                d2[e + 3 * WG] = a3;
            }
            for (; e < n2; e += WG) d2[e] = s2[e];
        } else {
            for (int64_t e = t; e < n; e += WG) dst[e] = src[e];
        }
        return;
    }
    const int mlo = mptr[li], k = mptr[li + 1] - mlo;
    // E_i's column list staged in LDS (one coalesced read), so that the k
    // position searches run in LDS instead of as chains of global loads
    constexpr int ECAP_U = NBT == 1 ? 64 : 512;
    __shared__ int32_t ecs[ECAP_U];
    const bool ecols = ek <= ECAP_U;   // uniform
    if (ecols)
        for (int q = t; q < ek; q += WG) ecs[q] = ecol[elo + q];
    __syncthreads();
    for (int p = t; p < k; p += WG) {
        const int32_t c = mcol[mlo + p];
        ncol[nlo + p] = c;
        if (k <= QCAP) {
            if (ecols) {
                const int r = bsearch_i32(ecs, 0, ek, c);
                qpos[p] = r < 0 ? -1 : elo + r;
            } else {
                qpos[p] = bsearch_i32(ecol, elo, elo + ek, c);
            }
        }
    }
    __syncthreads();
    const double *L = lamt + (int64_t)i * nb2;
    if constexpr (NBT > 1 && NBT % 2 == 0) {
        // Lambda~_i staged transposed (column u contiguous); each thread produces two
        // adjacent columns of an output block: per entry the same sum over u
        constexpr int NB2 = NBT * NBT, NH = NBT / 2;
        __shared__ __align__(16) double LT[MAXNB * MAXNB];
        for (int e = t; e < NB2; e += WG) LT[(e % NBT) * NBT + e / NBT] = L[e];
        __syncthreads();
        const double2 *lt2 = reinterpret_cast<const double2 *>(LT);
        for (int w = t; w < k * NH; w += WG) {
            const int p = w / NH, c2 = (w % NH) * 2;
            const int q = k <= QCAP ? qpos[p] : bsearch_i32(ecol, elo, elo + ek, mcol[mlo + p]);
            const double *mp = mval + (int64_t)(mlo + p) * NB2 + c2;
            double a0[NBT], a1[NBT];
#pragma unroll
            for (int r = 0; r < NBT; ++r) a0[r] = a1[r] = 0.0;
#pragma unroll 2
            for (int u = 0; u < NBT; ++u) {
                const double2 m = *reinterpret_cast<const double2 *>(mp + u * NBT);
#pragma unroll
                for (int r2 = 0; r2 < NH; ++r2) {
                    const double2 lv = lt2[u * NH + r2];
                    a0[2 * r2] += lv.x * m.x;
                    a0[2 * r2 + 1] += lv.y * m.x;
                    a1[2 * r2] += lv.x * m.y;
                    a1[2 * r2 + 1] += lv.y * m.y;
                }
            }
            double *no = nval + (int64_t)(nlo + p) * NB2 + c2;
            const double *eo = eval + (int64_t)(q >= 0 ? q : 0) * NB2 + c2;   // read only when q >= 0
#pragma unroll
            for (int r = 0; r < NBT; ++r) {
                const double2 v = q >= 0 ? *reinterpret_cast<const double2 *>(eo + r * NBT) : make_double2(0.0, 0.0);
                *reinterpret_cast<double2 *>(no + r * NBT) = make_double2(v.x - a0[r], v.y - a1[r]);
            }
        }
    } else if constexpr (NBT > 0 && WG % (NBT * NBT) == 0) {
        // each thread keeps one entry (r, sc) of the blocks and walks the blocks
        constexpr int NB2 = NBT * NBT, PER = WG / NB2;
        const int rs = t % NB2, r = rs / NBT, sc = rs % NBT;
        double lr[NBT];
#pragma unroll
        for (int u = 0; u < NBT; ++u) lr[u] = L[r * NBT + u];
        for (int p = t / NB2; p < k; p += PER) {
            const int q = k <= QCAP ? qpos[p] : bsearch_i32(ecol, elo, elo + ek, mcol[mlo + p]);
            const double v = (q >= 0) ? eval[(int64_t)q * NB2 + rs] : 0.0;
            const double *mp = mval + (int64_t)(mlo + p) * NB2 + sc;
            double m[NBT];
#pragma unroll
            for (int u = 0; u < NBT; ++u) m[u] = mp[u * NBT];
            double acc = 0.0;
#pragma unroll
            for (int u = 0; u < NBT; ++u) acc += lr[u] * m[u];
            nval[(int64_t)(nlo + p) * NB2 + rs] = v - acc;
        }
    } else {
        const int total = k * nb2;
        for (int e = t; e < total; e += WG) {
            const int p = e / nb2, rs = e % nb2;
            const int r = rs / nb, sc = rs % nb;
            const int q = k <= QCAP ? qpos[p] : bsearch_i32(ecol, elo, elo + ek, mcol[mlo + p]);
            const double v = (q >= 0) ? eval[(int64_t)q * nb2 + rs] : 0.0;
            const double *mp = mval + (int64_t)(mlo + p) * nb2 + sc;
            double acc = 0.0;
            for (int u = 0; u < nb; ++u) acc += L[r * nb + u] * mp[u * nb];
            nval[(int64_t)(nlo + p) * nb2 + rs] = v - acc;
        }
    }
}

void launch_eupdate(hipStream_t s, int B, int nb, const int32_t *pos, const int32_t *mptr, const int32_t *mcol,
                    const double *mval, const int32_t *eptr, const int32_t *ecol, const double *eval,
                    const double *lamt, const int32_t *nptr, int32_t *ncol, double *nval) {
    auto go = [&](auto nbc) {
        constexpr int NBT = decltype(nbc)::value;
        hipLaunchKernelGGL((k_eupdate<NBT>), dim3(B), dim3(WG), 0, s, B, nb, pos, mptr, mcol, mval, eptr, ecol, eval,
                           lamt, nptr, ncol, nval);
    };
    switch (nb) {
        case 1: go(std::integral_constant<int, 1>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        case 4: go(std::integral_constant<int, 4>{}); break;
        case 8: go(std::integral_constant<int, 8>{}); break;
        case 16: go(std::integral_constant<int, 16>{}); break;
        default: go(std::integral_constant<int, 0>{}); break;
    }
}

// Truncation: keep the alpha blocks of largest Frobenius norm of every list row
// (ties -> lower column).  COUNT pass writes the kept count, FILL copies.
template <bool FILL>
__global__ __launch_bounds__(WG) void k_truncate(int B, int nb, int alpha, const int32_t *__restrict__ pos_in_list,
                                                 const int32_t *__restrict__ eptr, const int32_t *__restrict__ ecol,
                                                 const double *__restrict__ eval, int32_t *__restrict__ cnt,
                                                 const int32_t *__restrict__ tptr, int32_t *__restrict__ tcol,
                                                 double *__restrict__ tval, int32_t *__restrict__ err) {
    __shared__ double nrm[UNION_CAP];
    __shared__ int32_t keep[UNION_CAP];
    const int i = blockIdx.x;
    if (i >= B) return;
    const int t = threadIdx.x;
    const int nb2 = nb * nb;
    const int elo = eptr[i], ek = eptr[i + 1] - elo;
    const bool trunc = pos_in_list[i] >= 0 && ek > alpha;
    if (!trunc) {
        if (!FILL) {
            if (t == 0) cnt[i] = ek;
        } else {
            const int tlo = tptr[i];
            for (int q = t; q < ek; q += WG) tcol[tlo + q] = ecol[elo + q];
            for (int64_t e = t; e < (int64_t)ek * nb2; e += WG)
                tval[(int64_t)tlo * nb2 + e] = eval[(int64_t)elo * nb2 + e];
        }
        return;
    }
    if (ek > UNION_CAP) {
        if (t == 0) {
            err[i] = 1;
            if (!FILL) cnt[i] = 0;
        }
        return;
    }
    if (!FILL) {
        if (t == 0) cnt[i] = alpha;
        return;
    }
    for (int q = t; q < ek; q += WG) {
        const double *ep = eval + (int64_t)(elo + q) * nb2;
        double s = 0.0;
        for (int e = 0; e < nb2; ++e) s += ep[e] * ep[e];
        nrm[q] = s;
    }
    __syncthreads();
    for (int q = t; q < ek; q += WG) {
        int rank = 0;
        double v = nrm[q];
        for (int u = 0; u < ek; ++u) {
            double o = nrm[u];
            rank += (o > v) || (o == v && u < q);
        }
        keep[q] = rank < alpha;
    }
    __syncthreads();
    if (t == 0) {
        int o = tptr[i], kept = 0;
        for (int q = 0; q < ek; ++q)
            if (keep[q] > 0 && kept < alpha) {
                ++kept;
                tcol[o] = ecol[elo + q];
                keep[q] = -(o + 1);
                ++o;
            }
    }
    __syncthreads();
    for (int64_t e = t; e < (int64_t)ek * nb2; e += WG) {
        int q = (int)(e / nb2), rs = (int)(e % nb2);
        int kq = keep[q];
        if (kq < 0) tval[(int64_t)(-kq - 1) * nb2 + rs] = eval[(int64_t)(elo + q) * nb2 + rs];
    }
}

__global__ void k_identity_E(int B, int nb, int32_t *ptr, int32_t *col, double *val) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t tot = (int64_t)B * nb * nb;
    if (e < B) {
        ptr[e] = (int32_t)e;
        col[e] = (int32_t)e;
    }
    if (e == 0) ptr[B] = B;
    if (e < tot) {
        int rs = (int)(e % (nb * nb));
        val[e] = (rs / nb == rs % nb) ? 1.0 : 0.0;
    }
}

__global__ void k_pos_in_list(const int32_t *__restrict__ list, int nlist, int32_t *__restrict__ pos) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nlist) pos[list[t]] = t;
}

__global__ void k_iota(int32_t *a, int n) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = t;
}

__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t v) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) a[t] = v;
}

// max over r < n of ptr[(r + 1) stride] - ptr[r stride] (out starts at 0)
__global__ __launch_bounds__(WG) void k_max_span(int64_t n, int stride, const int32_t *__restrict__ ptr,
                                                 int32_t *__restrict__ out) {
    __shared__ int32_t red[WG / 64];
    const int64_t r = blockIdx.x * (int64_t)WG + threadIdx.x;
    int32_t m = r < n ? ptr[(r + 1) * stride] - ptr[r * stride] : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < WG / 64; ++w) m = max(m, red[w]);
        atomicMax(out, m);
    }
}

// out += sum (SUM) or out = max(out, max) (!SUM) of a[0, n) (out starts at 0)
template <bool SUM>
__global__ __launch_bounds__(WG) void k_reduce_i32(int64_t n, const int32_t *__restrict__ a,
                                                   int32_t *__restrict__ out) {
    __shared__ int32_t red[WG / 64];
    int32_t m = 0;
    for (int64_t r = blockIdx.x * (int64_t)WG + threadIdx.x; r < n; r += (int64_t)gridDim.x * WG)
        m = SUM ? m + a[r] : max(m, a[r]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int32_t y = __shfl_xor(m, off, 64);
        m = SUM ? m + y : max(m, y);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < WG / 64; ++w) m = SUM ? m + red[w] : max(m, red[w]);
        if (SUM) atomicAdd(out, m);
        else atomicMax(out, m);
    }
}

// block-row lengths of the updated E: list rows take |pattern(M_i)|, the others keep |pattern(E_i)|
// (members of a lattice class, pos -2, take the length of their representative's new row)
__global__ void k_ecount(int B, const int32_t *__restrict__ pos, const int32_t *__restrict__ rep,
                         const int32_t *__restrict__ mptr, const int32_t *__restrict__ eptr,
                         int32_t *__restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    int q = pos[i];
    if (q == -2) q = pos[rep[i]];
    cnt[i] = q >= 0 ? mptr[q + 1] - mptr[q] : eptr[i + 1] - eptr[i];
}

// Reference smoother of Sec. 2.1 (damped block Jacobi; block Gauss-Seidel in
// multiplicative mode): Lambda_l = omega A_ii^{-1} for every cascade level l.
// One wavefront per block (four per workgroup): [A_ii | I] in LDS, gathered
// from the scalar CSR rows of the block, then Gauss-Jordan elimination with
// partial pivoting (the row of the largest |a_rk| at or below the pivot, the
// first on ties); the right half ends as the inverse.  A zero or non-finite
// pivot flags the block (bad[i] = 1, its Lambda zero).  Blocks at or beyond
// B_act (rows solved directly) get zero Lambda and are not checked.
__global__ __launch_bounds__(WG) void k_block_jacobi(int64_t B, int64_t B_act, int nb, int depth, double omega,
                                                     const int32_t *__restrict__ a_ptr,
                                                     const int32_t *__restrict__ a_col,
                                                     const double *__restrict__ a_val, double *__restrict__ lam,
                                                     int32_t *__restrict__ bad) {
    __shared__ double m[WG / 64][MAXNB * 2 * MAXNB];
    __shared__ double fac[WG / 64][MAXNB];
    __shared__ int piv[WG / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * (WG / 64) + wv;
    const bool act = i < B_act;   // uniform per wavefront; inactive ones still reach every barrier
    const int w2 = 2 * nb;
    double *a = m[wv];
    for (int e = lane; e < nb * w2; e += 64) {
        const int r = e / w2, q = e % w2;
        a[e] = (q - nb == r) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (act && lane < nb) {
        const int64_t row = i * nb + lane;
        for (int e = a_ptr[row]; e < a_ptr[row + 1]; ++e) {
            const int64_t cj = (int64_t)a_col[e] - i * nb;
            if (cj >= 0 && cj < nb) a[lane * w2 + cj] += a_val[e];
        }
    }
    __syncthreads();
    bool ok = act;
    for (int k = 0; k < nb; ++k) {
        if (lane == 0) {
            int p = k;
            double best = fabs(a[k * w2 + k]);
            for (int r = k + 1; r < nb; ++r) {
                const double v = fabs(a[r * w2 + k]);
                if (v > best) {
                    best = v;
                    p = r;
                }
            }
            piv[wv] = p;
        }
        __syncthreads();
        const int p = piv[wv];
        const double pv = a[p * w2 + k];
        ok = ok && pv != 0.0 && isfinite(pv);
        const double inv = (pv != 0.0 && isfinite(pv)) ? 1.0 / pv : 0.0;
        double tk = 0.0, tp = 0.0;
        if (lane < w2) {   // swap rows k and p, scale the pivot row
            tk = a[k * w2 + lane];
            tp = a[p * w2 + lane];
        }
        __syncthreads();
        if (lane < w2) {
            a[p * w2 + lane] = tk;
            a[k * w2 + lane] = tp * inv;
        }
        __syncthreads();
        if (lane < nb) fac[wv][lane] = a[lane * w2 + k];
        __syncthreads();
        for (int e = lane; e < nb * w2; e += 64) {
            const int r = e / w2, q = e % w2;
            if (r != k) a[e] -= fac[wv][r] * a[k * w2 + q];
        }
        __syncthreads();
    }
    if (i < B) {
        if (act && !ok && lane == 0) bad[i] = 1;
        const int64_t nb2 = (int64_t)nb * nb;
        for (int e = lane; e < nb * nb; e += 64) {
            const int r = e / nb, q = e % nb;
            const double v = (act && ok) ? omega * a[r * w2 + nb + q] : 0.0;
            for (int ell = 0; ell < depth; ++ell) lam[((int64_t)ell * B + i) * nb2 + e] = v;
        }
    }
}

__global__ void k_unscale(int64_t B, int nb, const double *__restrict__ w, const double *__restrict__ lamt,
                          double *__restrict__ lam) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int nb2 = nb * nb;
    if (e >= B * nb2) return;
    int64_t i = e / nb2;
    int rs = (int)(e % nb2), r = rs / nb, s = rs % nb;
    lam[e] = w[i * nb + r] * lamt[e] * w[i * nb + s];
}

// Lambda[ell][i] = W_i Lambda~[i][ell] W_i from the network's FP32 layout
// [B][depth][nb][nb] into the FP64 master [depth][B][nb][nb]
__global__ void k_unscale_learned(int64_t B, int nb, int depth, const double *__restrict__ w,
                                  const float *__restrict__ lt, double *__restrict__ lam) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int nb2 = nb * nb;
    if (e >= (int64_t)depth * B * nb2) return;
    const int ell = (int)(e / (B * nb2));
    const int64_t rem = e % (B * nb2);
    const int64_t i = rem / nb2;
    const int rs = (int)(rem % nb2), r = rs / nb, c = rs % nb;
    lam[e] = w[i * nb + r] * (double)lt[(i * depth + ell) * nb2 + rs] * w[i * nb + c];
}

// Lambda~ = W^-1 Lambda W^-1 in the network's layout [B][depth][nb][nb]
__global__ void k_prescaled_export(int64_t B, int nb, int depth, const double *__restrict__ w,
                                   const double *__restrict__ lam, float *__restrict__ out) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int nb2 = nb * nb;
    if (e >= (int64_t)depth * B * nb2) return;
    const int64_t i = e / ((int64_t)depth * nb2);
    const int64_t rem = e % ((int64_t)depth * nb2);
    const int ell = (int)(rem / nb2);
    const int rs = (int)(rem % nb2), r = rs / nb, c = rs % nb;
    out[e] = (float)(lam[((int64_t)ell * B + i) * nb2 + rs] / (w[i * nb + r] * w[i * nb + c]));
}

// ---------------------------------------------------------------------------
// colouring
// ---------------------------------------------------------------------------

// One round of greedy colouring in block-index order: a block takes the smallest
// colour unused by its lower-index neighbours once all of those are coloured.
// Produces exactly the sequential greedy colouring.
__global__ __launch_bounds__(WG) void k_greedy_round(int B, const int32_t *__restrict__ bptr,
                                                     const int32_t *__restrict__ bcol, int32_t *colour,
                                                     int32_t *__restrict__ pending) {
    const int i = blockIdx.x * WG + threadIdx.x;
    int waiting = 0;
    if (i < B && colour[i] < 0) {
        uint64_t used = 0;   // colours 0..63
        bool ready = true, overflow = false;
        for (int k = bptr[i]; k < bptr[i + 1]; ++k) {
            int j = bcol[k];
            if (j >= i) continue;
            int cj = __atomic_load_n(&colour[j], __ATOMIC_RELAXED);
            if (cj < 0) {
                ready = false;
                break;
            }
            if (cj < 64) used |= (1ull << cj);
            else overflow = true;
        }
        if (ready && !overflow) {
            int cbit = __builtin_ctzll(~used);
            __atomic_store_n(&colour[i], cbit, __ATOMIC_RELAXED);
        } else {
            waiting = 1;
        }
    }
    int any = __syncthreads_or(waiting);
    if (threadIdx.x == 0) pending[blockIdx.x] = any;
}

__global__ void k_colour_check(int B, const int32_t *__restrict__ bptr, const int32_t *__restrict__ bcol,
                               const int32_t *__restrict__ colour, int32_t *__restrict__ bad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    int ci = colour[i], b = 0;
    for (int k = bptr[i]; k < bptr[i + 1]; ++k) {
        int j = bcol[k];
        if (j != i && colour[j] == ci) b = 1;
    }
    bad[i] = b;
}

// ---------------------------------------------------------------------------
// bottom level: Gauss-Jordan inversion, one pivot per launch (ping-pong)
// ---------------------------------------------------------------------------
__global__ void k_gauss_jordan(const double *__restrict__ in, double *__restrict__ out, int n, int k) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    int i = (int)(e / n), j = (int)(e % n);
    double p = in[(int64_t)k * n + k];
    double v;
    if (i == k) v = (j == k) ? 1.0 / p : in[(int64_t)k * n + j] / p;
    else {
        double f = in[(int64_t)i * n + k];
        v = (j == k) ? -f / p : in[e] - f * in[(int64_t)k * n + j] / p;
    }
    out[e] = v;
}

// One Gauss-Jordan pivot step k applied to every segment's dense matrix at
// once; segments already past their size are copied unchanged.
// One Gauss-Jordan step k on the segments that are still active: segments are
// packed largest first, so the active ones are a prefix [0, nact) and their
// entries the range [0, soff[nact]).  Segment q is m[q] x m[q], row-major.
__global__ void k_gauss_jordan_seg(const double *__restrict__ in, double *__restrict__ out, int nact,
                                   const int64_t *__restrict__ soff, const int32_t *__restrict__ msz, int k) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= soff[nact]) return;
    int lo = 0, hi = nact;   // segment q with soff[q] <= e < soff[q+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (soff[mid] <= e) lo = mid;
        else hi = mid;
    }
    const int64_t base = soff[lo];
    const int m = msz[lo];
    const int loc = (int)(e - base), i = loc / m, j = loc % m;
    const double *a = in + base;
    const double p = a[k * m + k];
    double v;
    if (i == k) v = (j == k) ? 1.0 / p : a[k * m + j] / p;
    else {
        const double f = a[i * m + k];
        v = (j == k) ? -f / p : a[loc] - f * a[k * m + j] / p;
    }
    out[e] = v;
}

// Final inverses into their places: packed segment q finished in buffer b1
// when its size is odd (steps alternate a -> b -> a ...), else in b0.
__global__ void k_gauss_jordan_collect(int64_t tot, int nseg, const int64_t *__restrict__ soff,
                                       const int32_t *__restrict__ msz, const int64_t *__restrict__ dst_off,
                                       const double *__restrict__ b0, const double *__restrict__ b1,
                                       double *__restrict__ out) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= tot) return;
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (soff[mid] <= e) lo = mid;
        else hi = mid;
    }
    out[dst_off[lo] + (e - soff[lo])] = (msz[lo] & 1) ? b1[e] : b0[e];
}

__global__ void k_transpose_blocks64(int64_t nblk, int nb, const double *__restrict__ a, double *__restrict__ at) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int nb2 = nb * nb;
    if (e >= nblk * nb2) return;
    int64_t i = e / nb2;
    int rs = (int)(e % nb2), r = rs / nb, s = rs % nb;
    at[i * nb2 + s * nb + r] = a[e];
}

__global__ void k_cast32(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) b[e] = (float)a[e];
}

// ---------------------------------------------------------------------------
// Stencil-repetition cache (Sec. 4): blocks at integer lattice points whose
// neighbourhoods coincide under translation share one cascade fit.  Classes
// are refined one block layer per round: round 0 compares the block rows of A
// (offsets to the block columns, the stored values, the diagonals of the
// column blocks), round r the class of the row at round r - 1 and those of
// its neighbours, by offset.  A 64-bit key per block finds a candidate (the
// smallest block with the same key, through an open-addressing table); the
// candidate is then checked exactly, so a key collision can only make a block
// its own representative (a lost share), never a wrong one.  The constants
// mixed into the keys are arbitrary odd 64-bit words that keep the inputs
// (offsets, positions, values, classes) apart.
// ---------------------------------------------------------------------------
struct LatDev {
    const int32_t *xyz;   // [B][3] lattice points (unused axes 0)
    const int32_t *map;   // bounding box point -> block, -1 where none
    int32_t lo0, lo1, lo2, ex0, ex1, ex2;
};

constexpr uint64_t LAT_EMPTY = ~0ull;
constexpr int LAT_ROW_CAP = 2048;   // blocks per residual row that the translation copy holds in LDS

// SplitMix64 output mixing (Steele, Lea and Flood, 2014)
__device__ inline uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ull;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ inline uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }

__device__ inline uint64_t lat_offset_key(const LatDev &L, int c, int k) {
    const int32_t *pc = L.xyz + 3 * (int64_t)c, *pk = L.xyz + 3 * (int64_t)k;
    return mix64(((uint64_t)(uint32_t)(pc[0] - pk[0])) ^ ((uint64_t)(uint32_t)(pc[1] - pk[1]) << 21) ^
                 ((uint64_t)(uint32_t)(pc[2] - pk[2]) << 42));
}

// block at the lattice point of c moved by xyz[to] - xyz[from], or -1
__device__ inline int lat_shift(const LatDev &L, int c, int from, int to) {
    const int32_t *pc = L.xyz + 3 * (int64_t)c, *pf = L.xyz + 3 * (int64_t)from, *pt = L.xyz + 3 * (int64_t)to;
    const int x = pc[0] - pf[0] + pt[0] - L.lo0, y = pc[1] - pf[1] + pt[1] - L.lo1, z = pc[2] - pf[2] + pt[2] - L.lo2;
    if ((unsigned)x >= (unsigned)L.ex0 || (unsigned)y >= (unsigned)L.ex1 || (unsigned)z >= (unsigned)L.ex2) return -1;
    return L.map[((int64_t)z * L.ex1 + y) * L.ex0 + x];
}

__device__ inline uint64_t lat_fix(uint64_t h) { return h == LAT_EMPTY ? h - 1 : h; }

__device__ inline int lat_lookup(uint64_t h, int64_t T, const uint64_t *__restrict__ tk, const int32_t *__restrict__ tm) {
    int64_t s = (int64_t)(h & (uint64_t)(T - 1));
    while (tk[s] != h) s = (s + 1) & (T - 1);   // the key was inserted: the probe ends there
    return tm[s];
}

__global__ void k_lat_diag(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           const double *__restrict__ val, double *__restrict__ diag) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int q = bsearch_i32(col, ptr[r], ptr[r + 1], (int32_t)r);
    diag[r] = q >= 0 ? val[q] : 0.0;
}

// round 0 key: block columns (offset, diagonals) and stored non-zero-bit entries
// (offset, position in the block, value); a stored +0.0 counts as absent
__global__ void k_lat_key0(int B, int nb, const int32_t *__restrict__ bptr, const int32_t *__restrict__ bcol,
                           const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           const double *__restrict__ val, const double *__restrict__ diag, LatDev L,
                           uint64_t *__restrict__ key) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B) return;
    uint64_t h = mix64((uint64_t)(bptr[k + 1] - bptr[k]));
    for (int e = bptr[k]; e < bptr[k + 1]; ++e) {
        const int c = bcol[e];
        uint64_t t = lat_offset_key(L, c, k);
        for (int s = 0; s < nb; ++s) t = mix64(t ^ dbits(diag[(int64_t)c * nb + s]));
        h += t;
    }
    for (int q = 0; q < nb; ++q) {
        const int64_t r = (int64_t)k * nb + q;
        for (int e = ptr[r]; e < ptr[r + 1]; ++e) {
            const uint64_t v = dbits(val[e]);
            if (!v) continue;
            const int j = col[e];
            h += mix64(lat_offset_key(L, j / nb, k) ^ mix64(0x9e3779b97f4a7c15ull * (uint64_t)(q * nb + j % nb + 1)) ^
                       v);
        }
    }
    key[k] = lat_fix(mix64(h));
}

// round r > 0 key: own class and the classes of the neighbours, by offset
__global__ void k_lat_key(int B, const int32_t *__restrict__ bptr, const int32_t *__restrict__ bcol, LatDev L,
                          const int32_t *__restrict__ prev, uint64_t *__restrict__ key) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B) return;
    uint64_t h = mix64((uint64_t)prev[k] + 0x632be59bd9b4e019ull);
    for (int e = bptr[k]; e < bptr[k + 1]; ++e) {
        const int c = bcol[e];
        h += mix64(lat_offset_key(L, c, k) ^ (uint64_t)(uint32_t)prev[c]);
    }
    key[k] = lat_fix(mix64(h));
}

__global__ void k_lat_clear(int64_t T, uint64_t *__restrict__ tk, int32_t *__restrict__ tm) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= T) return;
    tk[s] = LAT_EMPTY;
    tm[s] = INT32_MAX;
}

// T > 2B slots: a free slot is always met, so the probe ends.  Neighbouring
// blocks mostly share a key, so a wavefront first reduces its lanes per key
// and one lane inserts each distinct key with the smallest block.
__global__ __launch_bounds__(WG) void k_lat_insert(int B, const uint64_t *__restrict__ key, int64_t T,
                                                   uint64_t *__restrict__ tk, int32_t *__restrict__ tm) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool active = k < B;
    const uint64_t h = active ? key[k] : 0;
    uint64_t pending = __ballot(active);
    while (pending) {   // wavefront-uniform
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const uint64_t hl = __shfl(h, leader, 64);
        const bool mine = ((pending >> lane) & 1) && h == hl;
        int v = mine ? k : INT32_MAX;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
        if (lane == leader) {
            int64_t s = (int64_t)(hl & (uint64_t)(T - 1));
            for (;;) {
                const unsigned long long prev = atomicCAS((unsigned long long *)(tk + s),
                                                          (unsigned long long)LAT_EMPTY, (unsigned long long)hl);
                if (prev == LAT_EMPTY || prev == hl) {
                    atomicMin(tm + s, v);
                    break;
                }
                s = (s + 1) & (T - 1);
            }
        }
        pending &= ~__ballot(mine);
    }
}

// same block pattern under the translation k -> r (and, for rounds > 0, the same
// classes of the neighbours)
__device__ inline bool lat_same_blocks(int k, int r, const int32_t *__restrict__ bptr,
                                       const int32_t *__restrict__ bcol, const LatDev &L,
                                       const int32_t *__restrict__ prev) {
    if (bptr[k + 1] - bptr[k] != bptr[r + 1] - bptr[r]) return false;
    for (int e = bptr[k]; e < bptr[k + 1]; ++e) {
        const int c = bcol[e];
        const int c2 = lat_shift(L, c, k, r);
        if (c2 < 0 || bsearch_i32(bcol, bptr[r], bptr[r + 1], c2) < 0) return false;
        if (prev && prev[c] != prev[c2]) return false;
    }
    return true;
}

__global__ void k_lat_rep0(int B, int nb, const int32_t *__restrict__ bptr, const int32_t *__restrict__ bcol,
                           const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           const double *__restrict__ val, const double *__restrict__ diag, LatDev L,
                           const uint64_t *__restrict__ key, int64_t T, const uint64_t *__restrict__ tk,
                           const int32_t *__restrict__ tm, int32_t *__restrict__ rep) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B) return;
    const int r = lat_lookup(key[k], T, tk, tm);
    bool ok = r != k && lat_same_blocks(k, r, bptr, bcol, L, nullptr);
    for (int e = bptr[k]; ok && e < bptr[k + 1]; ++e) {
        const int c = bcol[e], c2 = lat_shift(L, c, k, r);
        for (int s = 0; s < nb; ++s)
            ok = ok && dbits(diag[(int64_t)c * nb + s]) == dbits(diag[(int64_t)c2 * nb + s]);
    }
    for (int q = 0; ok && q < nb; ++q) {
        const int64_t rk = (int64_t)k * nb + q, rr = (int64_t)r * nb + q;
        int nk = 0, nr = 0;
        for (int e = ptr[rk]; e < ptr[rk + 1]; ++e) nk += dbits(val[e]) != 0;
        for (int e = ptr[rr]; e < ptr[rr + 1]; ++e) nr += dbits(val[e]) != 0;
        ok = nk == nr;
        for (int e = ptr[rk]; ok && e < ptr[rk + 1]; ++e) {
            const uint64_t v = dbits(val[e]);
            if (!v) continue;
            const int j = col[e];
            const int c2 = lat_shift(L, j / nb, k, r);
            const int p = c2 < 0 ? -1 : bsearch_i32(col, ptr[rr], ptr[rr + 1], c2 * nb + j % nb);
            ok = p >= 0 && dbits(val[p]) == v;
        }
    }
    rep[k] = ok ? r : k;
}

__global__ void k_lat_rep(int B, const int32_t *__restrict__ bptr, const int32_t *__restrict__ bcol, LatDev L,
                          const int32_t *__restrict__ prev, const uint64_t *__restrict__ key, int64_t T,
                          const uint64_t *__restrict__ tk, const int32_t *__restrict__ tm,
                          int32_t *__restrict__ rep) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B) return;
    const int r = lat_lookup(key[k], T, tk, tm);
    const bool ok = r != k && prev[k] == prev[r] && lat_same_blocks(k, r, bptr, bcol, L, prev);
    rep[k] = ok ? r : k;
}

__global__ void k_lat_flag(int B, const int32_t *__restrict__ rep, int32_t *__restrict__ flag) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < B) flag[k] = rep[k] == k;
}

__global__ void k_lat_compact(int B, const int32_t *__restrict__ rep, const int32_t *__restrict__ off,
                              int32_t *__restrict__ list) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < B && rep[k] == k) list[off[k]] = k;
}

// members of a class (rep != self) are marked -2 in pos_in_list
__global__ void k_lat_mark(int B, const int32_t *__restrict__ rep, int32_t *__restrict__ pos) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < B && rep[k] != k) pos[k] = -2;
}

// Lambda~ of members from their representative; msing[k] = 1 for a member whose
// representative took the pseudo-inverse fallback
__global__ void k_lat_copy_lam(int B, int nb2, const int32_t *__restrict__ rep, const int32_t *__restrict__ pos,
                               const int32_t *__restrict__ sing, double *__restrict__ lam,
                               int32_t *__restrict__ msing) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * nb2) return;
    const int k = (int)(e / nb2), rs = (int)(e % nb2);
    const int r = rep[k];
    if (r == k) {
        if (rs == 0) msing[k] = 0;
        return;
    }
    lam[e] = lam[(int64_t)r * nb2 + rs];
    if (rs == 0) msing[k] = sing[pos[r]];
}

// need[c] = 1 for the blocks of the next step's list and their neighbours: the
// only rows whose residual values the next step reads
__global__ void k_lat_need(int nl, const int32_t *__restrict__ list, const int32_t *__restrict__ bptr,
                           const int32_t *__restrict__ bcol, int32_t *__restrict__ need) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nl) return;
    const int i = list[t];
    for (int e = bptr[i]; e < bptr[i + 1]; ++e) need[bcol[e]] = 1;
}

// Residual row of a member: the representative's new row with its block
// columns moved by the translation, re-sorted by rank; the values only where
// need[i] is set (need = NULL: everywhere).
__global__ __launch_bounds__(WG) void k_lat_etranslate(int B, int nb, const int32_t *__restrict__ pos,
                                                       const int32_t *__restrict__ rep, LatDev L,
                                                       const int32_t *__restrict__ need,
                                                       const int32_t *__restrict__ nptr, int32_t *__restrict__ ncol,
                                                       double *__restrict__ nval, int32_t *__restrict__ err) {
    __shared__ int32_t tc[LAT_ROW_CAP];
    __shared__ int32_t rk[LAT_ROW_CAP];
    const int i = blockIdx.x;
    if (i >= B || pos[i] != -2) return;
    const int r = rep[i];
    const int rlo = nptr[r], k = nptr[r + 1] - rlo, ilo = nptr[i];
    const int nb2 = nb * nb;
    if (k > LAT_ROW_CAP || k != nptr[i + 1] - ilo) {   // fails the setup; keep the columns valid meanwhile
        if (threadIdx.x == 0) err[i] = 1;
        for (int p = threadIdx.x; p < nptr[i + 1] - ilo; p += WG) ncol[ilo + p] = i;
        return;
    }
    for (int p = threadIdx.x; p < k; p += WG) {
        int c = lat_shift(L, ncol[rlo + p], r, i);
        if (c < 0) {   // cannot happen for verified classes; keep later indexing in bounds until the check
            err[i] = 1;
            c = i;
        }
        tc[p] = c;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < k; p += WG) {
        const int v = tc[p];
        int below = 0;
        for (int q = 0; q < k; ++q) below += tc[q] < v;
        rk[p] = below;
        ncol[ilo + below] = v;
    }
    if (need && !need[i]) return;   // block-uniform
    __syncthreads();
    const bool fixed = WG % nb2 == 0;
    const int total = k * nb2;
    for (int e0 = 0; e0 < total; e0 += WG) {
        const int e = e0 + (int)threadIdx.x;
        if (e >= total) break;
        const int p = fixed ? e0 / nb2 + (int)threadIdx.x / nb2 : e / nb2;
        const int rs = fixed ? (int)threadIdx.x % nb2 : e % nb2;
        nval[(int64_t)(ilo + rk[p]) * nb2 + rs] = nval[(int64_t)(rlo + p) * nb2 + rs];
    }
}

inline unsigned grid_for(int64_t n, int wg = WG) { return (unsigned)ceil_div(n, wg); }

struct EMat {
    BPattern pat;
    DBuf<double> val;
};

int64_t scan_counts(Ctx &c, const DBuf<int32_t> &cnt, int64_t n, DBuf<int32_t> &ptr, DBuf<int64_t> &tot) {
    ptr.alloc(n + 1);
    const int64_t ntiles = std::max<int64_t>(ceil_div(n, SCAN_TILE), 1);
    DBuf<int64_t> tiles(ntiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(256), 0, c.stream, cnt.get(), n, ptr.get(),
                       tiles.get());
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, c.stream, ntiles, tiles.get(), tot.get());
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)ceil_div(n + 1, 256)), dim3(256), 0, c.stream, n, tiles.get(),
                       tot.get(), ptr.get());
    CS_LAUNCH_CHECK();
    int64_t total = 0;
    tot.download(&total, 1, c.stream);
    CS_HIP(hipStreamSynchronize(c.stream));
    if (total >= INT32_MAX) fail(CS_ENOMEM, "pattern too large for 32-bit offsets");
    return total;
}

// scan_counts that also brings back, in the same round trip, max(cnt[0, n))
// (when maxc) and max(flags[0, nflags)) (when flags)
int64_t scan_counts_ex(Ctx &c, const DBuf<int32_t> &cnt, int64_t n, DBuf<int32_t> &ptr, DBuf<int64_t> &tot,
                       int32_t *maxc, const int32_t *flags, int64_t nflags, int32_t *flag) {
    DBuf<int32_t> m(2);
    hipStream_t s = c.stream;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(WG), 0, s, m.get(), (int64_t)2, 0);
    if (maxc && n > 0)
        hipLaunchKernelGGL(k_reduce_i32<false>, dim3((unsigned)std::min<int64_t>(ceil_div(n, WG), 4096)), dim3(WG), 0,
                           s, n, cnt.get(), m.get());
    if (flags && nflags > 0)
        hipLaunchKernelGGL(k_reduce_i32<false>, dim3((unsigned)std::min<int64_t>(ceil_div(nflags, WG), 4096)),
                           dim3(WG), 0, s, nflags, flags, m.get() + 1);
    ptr.alloc(n + 1);
    const int64_t ntiles = std::max<int64_t>(ceil_div(n, SCAN_TILE), 1);
    DBuf<int64_t> tiles(ntiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(256), 0, s, cnt.get(), n, ptr.get(), tiles.get());
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, ntiles, tiles.get(), tot.get());
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)ceil_div(n + 1, 256)), dim3(256), 0, s, n, tiles.get(), tot.get(),
                       ptr.get());
    CS_LAUNCH_CHECK();
    int64_t total = 0;
    int32_t hm[2] = {0, 0};
    tot.download(&total, 1, s);
    m.download(hm, 2, s);
    CS_HIP(hipStreamSynchronize(s));
    if (maxc) *maxc = hm[0];
    if (flag) *flag = hm[1];
    if (total >= INT32_MAX) fail(CS_ENOMEM, "pattern too large for 32-bit offsets");
    return total;
}

// sum (or max) of n device ints, on the host
int32_t reduce_i32(Ctx &c, const int32_t *a, int64_t n, bool sum) {
    DBuf<int32_t> m(1);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(WG), 0, c.stream, m.get(), (int64_t)1, 0);
    const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(ceil_div(n, WG), 1), 4096);
    if (sum) hipLaunchKernelGGL(k_reduce_i32<true>, dim3(g), dim3(WG), 0, c.stream, n, a, m.get());
    else hipLaunchKernelGGL(k_reduce_i32<false>, dim3(g), dim3(WG), 0, c.stream, n, a, m.get());
    CS_LAUNCH_CHECK();
    int32_t h = 0;
    m.download(&h, 1, c.stream);
    CS_HIP(hipStreamSynchronize(c.stream));
    return h;
}

void check_flags(Ctx &c, const DBuf<int32_t> &flags, int64_t n, const char *what) {
    if (reduce_i32(c, flags.get(), n, false))
        fail(CS_EINVAL, std::string(what) + " exceeds the per-row capacity of the symbolic kernels");
}

}  // namespace

// ---------------------------------------------------------------------------
// host-side layout builders
// ---------------------------------------------------------------------------

void build_sell(Sell &S, const std::vector<int64_t> &ptr, const std::vector<int32_t> &col,
                const std::vector<double> &val, const std::vector<int32_t> *rows, hipStream_t s,
                bool pad_with_row) {
    const int64_t m = rows ? (int64_t)rows->size() : (int64_t)ptr.size() - 1;
    S.nrows = m;
    S.nslices = ceil_div(m, 64);
    std::vector<int64_t> sp(S.nslices + 1, 0);
    std::vector<int32_t> sl(S.nslices, 0);
    for (int64_t sidx = 0; sidx < S.nslices; ++sidx) {
        int len = 0;
        for (int l = 0; l < 64; ++l) {
            int64_t q = sidx * 64 + l;
            if (q >= m) break;
            int64_t r = rows ? (*rows)[q] : q;
            len = std::max<int>(len, (int)(ptr[r + 1] - ptr[r]));
        }
        sl[sidx] = len;
        sp[sidx + 1] = sp[sidx] + (int64_t)len * 64;
    }
    S.entries = sp[S.nslices];
    S.nnz = 0;
    for (int64_t q = 0; q < m; ++q) {
        int64_t r = rows ? (*rows)[q] : q;
        S.nnz += ptr[r + 1] - ptr[r];
    }
    std::vector<int32_t> hc(S.entries);
    std::vector<double> hv(S.entries);
    for (int64_t sidx = 0; sidx < S.nslices; ++sidx)
        for (int l = 0; l < 64; ++l) {
            int64_t q = sidx * 64 + l;
            int64_t r = (q < m) ? (rows ? (*rows)[q] : q) : -1;
            int64_t rl = r >= 0 ? ptr[r + 1] - ptr[r] : 0;
            for (int k = 0; k < sl[sidx]; ++k) {
                int64_t o = sp[sidx] + (int64_t)k * 64 + l;
                if (k < rl) {
                    hc[o] = col[ptr[r] + k];
                    hv[o] = val[ptr[r] + k];
                } else {   // padding: a zero at the row's own index (square A) or at column 0
                    hc[o] = (pad_with_row && r >= 0) ? (int32_t)r : 0;
                    hv[o] = 0.0;
                }
            }
        }
    S.slice_ptr.upload(sp.data(), sp.size(), s);
    S.slice_len.upload(sl.data(), sl.size(), s);
    S.col.upload(hc.data(), hc.size(), s);
    S.val64.upload(hv.data(), hv.size(), s);
    std::vector<float> hf(hv.begin(), hv.end());
    S.val32.upload(hf.data(), hf.size(), s);
    if (rows) {
        std::vector<int32_t> hr(S.nslices * 64, -1);
        for (int64_t q = 0; q < m; ++q) hr[q] = (*rows)[q];
        S.rows.upload(hr.data(), hr.size(), s);
    } else {
        S.rows.release();
    }
    CS_HIP(hipStreamSynchronize(s));   // host staging vectors go out of scope
}

void build_level_device(Ctx &c, Level &L) {
    hipStream_t s = c.stream;
    std::vector<int32_t> p32(L.h_ptr.begin(), L.h_ptr.end());
    L.a_ptr.upload(p32.data(), p32.size(), s);
    L.a_col.upload(L.h_col.data(), L.h_col.size(), s);
    L.a_val.upload(L.h_val.data(), L.h_val.size(), s);
    build_sell(L.sell, L.h_ptr, L.h_col, L.h_val, nullptr, s);
    L.act_slices = ceil_div(L.n_active, 64);
    L.act_nnz = L.h_ptr[L.n_active];
    // direct segments: offsets of their dense inverses in dinv
    const int nseg = (int)L.dseg.size() - 1;
    if (nseg > 0) {
        std::vector<int64_t> off(nseg + 1, 0);
        L.dseg_max = 0;
        for (int k = 0; k < nseg; ++k) {
            const int64_t m = L.dseg[k + 1] - L.dseg[k];
            off[k + 1] = off[k] + m * m;
            L.dseg_max = std::max(L.dseg_max, m);
        }
        L.dseg_d.upload(L.dseg.data(), L.dseg.size(), s);
        L.dinv_off.upload(off.data(), off.size(), s);
        L.dinv.alloc(off[nseg]);
    } else {
        L.dseg_max = 0;
        L.dinv.release();
    }
    CS_HIP(hipStreamSynchronize(s));
    build_bf16_level(c, L);
}

void build_colour_layout(Ctx &c, Level &L) {
    // blocks sorted by colour (stable), per-colour SELL over their scalar rows
    const int chi = 1 + *std::max_element(L.h_colour.begin(), L.h_colour.end());
    L.chi = chi;
    L.cptr.assign(chi + 1, 0);
    for (int32_t v : L.h_colour) L.cptr[v + 1]++;
    for (int k = 0; k < chi; ++k) L.cptr[k + 1] += L.cptr[k];
    std::vector<int32_t> list(L.B);
    std::vector<int64_t> fillp(L.cptr.begin(), L.cptr.end() - 1);
    for (int64_t i = 0; i < L.B; ++i) list[fillp[L.h_colour[i]]++] = (int32_t)i;
    L.clist.upload(list.data(), list.size(), c.stream);
    L.csell.clear();
    L.csell.resize(chi);
    std::vector<int32_t> act;                 // active blocks by colour
    L.cblk_ptr.assign(chi + 1, 0);
    for (int k = 0; k < chi; ++k) {
        for (int64_t q = L.cptr[k]; q < L.cptr[k + 1]; ++q)
            if (list[q] * L.nb < L.n_active) act.push_back(list[q]);
        L.cblk_ptr[k + 1] = (int64_t)act.size();
    }
    L.cblk.upload(act.data(), act.size(), c.stream);
    build_bf16_meta(c, L, act);
    for (int k = 0; k < chi; ++k) {
        std::vector<int32_t> rows;
        rows.reserve((L.cptr[k + 1] - L.cptr[k]) * L.nb);
        for (int64_t q = L.cptr[k]; q < L.cptr[k + 1]; ++q)
            if (list[q] * L.nb < L.n_active)   // rows of direct segments are not smoothed
                for (int r = 0; r < L.nb; ++r) rows.push_back((int32_t)(list[q] * L.nb + r));
        build_sell(L.csell[k], L.h_ptr, L.h_col, L.h_val, &rows, c.stream);
    }
    CS_HIP(hipStreamSynchronize(c.stream));
}

// ---------------------------------------------------------------------------
// setup driver
// ---------------------------------------------------------------------------

namespace {

int max_span(Ctx &c, int64_t n, int stride, const int32_t *ptr) {
    DBuf<int32_t> m(1);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(WG), 0, c.stream, m.get(), (int64_t)1, 0);
    hipLaunchKernelGGL(k_max_span, dim3(grid_for(std::max<int64_t>(n, 1))), dim3(WG), 0, c.stream, n, stride, ptr,
                       m.get());
    CS_LAUNCH_CHECK();
    int32_t h = 0;
    m.download(&h, 1, c.stream);
    CS_HIP(hipStreamSynchronize(c.stream));
    return h;
}

// Union of sorted column lists for nl rows: one wavefront per row when every
// row has at most 512 candidates (the bound is an upper bound of the candidate
// count), else one workgroup per row (with the larger LDS buffer beyond 4096).
template <int SRC, bool FILL>
void launch_union(hipStream_t s, int64_t bound, const int32_t *list, int nl, int nb, const int32_t *sptr,
                  const int32_t *scol, const int32_t *eptr, const int32_t *ecol, int32_t *cnt, const int32_t *optr,
                  int32_t *ocol, int32_t *err) {
    const dim3 gw((unsigned)ceil_div(nl, WG / 64));
    if (bound <= 64)
        hipLaunchKernelGGL((k_union_wave<1, SRC, FILL>), gw, dim3(WG), 0, s, list, nl, nb, sptr, scol, eptr, ecol,
                           cnt, optr, ocol, err);
    else if (bound <= 128)
        hipLaunchKernelGGL((k_union_wave<2, SRC, FILL>), gw, dim3(WG), 0, s, list, nl, nb, sptr, scol, eptr, ecol,
                           cnt, optr, ocol, err);
    else if (bound <= 256)
        hipLaunchKernelGGL((k_union_wave<4, SRC, FILL>), gw, dim3(WG), 0, s, list, nl, nb, sptr, scol, eptr, ecol,
                           cnt, optr, ocol, err);
    else if (bound <= 512)
        hipLaunchKernelGGL((k_union_wave<8, SRC, FILL>), gw, dim3(WG), 0, s, list, nl, nb, sptr, scol, eptr, ecol,
                           cnt, optr, ocol, err);
    else if (bound <= UNION_CAP)
        hipLaunchKernelGGL((k_union<SRC, FILL>), dim3(nl), dim3(WG), 0, s, list, nl, nb, sptr, scol, eptr, ecol, cnt,
                           optr, ocol, err);
    else
        hipLaunchKernelGGL((k_union<SRC, FILL, UNION_CAP_BIG>), dim3(nl), dim3(WG), 0, s, list, nl, nb, sptr, scol,
                           eptr, ecol, cnt, optr, ocol, err);
}

void block_pattern_of_A(Ctx &c, Level &L, BPattern &ap) {
    const int B = (int)L.B;
    DBuf<int32_t> cnt(B), err(B);
    DBuf<int64_t> tot(1);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(B)), dim3(WG), 0, c.stream, err.get(), (int64_t)B, 0);
    const int64_t bound = max_span(c, B, (int)L.nb, L.a_ptr.get());
    launch_union<SRC_SCALAR, false>(c.stream, bound, nullptr, B, (int)L.nb, L.a_ptr.get(), L.a_col.get(), nullptr,
                                    nullptr, cnt.get(), nullptr, nullptr, err.get());
    CS_LAUNCH_CHECK();
    check_flags(c, err, B, "block row of A");
    ap.rows = B;
    ap.nnzb = scan_counts(c, cnt, B, ap.ptr, tot);
    ap.col.alloc(ap.nnzb);
    launch_union<SRC_SCALAR, true>(c.stream, bound, nullptr, B, (int)L.nb, L.a_ptr.get(), L.a_col.get(), nullptr,
                                   nullptr, nullptr, ap.ptr.get(), ap.col.get(), err.get());
    CS_LAUNCH_CHECK();
}

void greedy_colouring(Ctx &c, Level &L, const BPattern &ap) {
    const int B = (int)L.B;
    DBuf<int32_t> col(B), pend(grid_for(B));
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(B)), dim3(WG), 0, c.stream, col.get(), (int64_t)B, -1);
    std::vector<int32_t> hp(grid_for(B));
    for (int round = 0; round < B + 64; round += 16) {
        for (int q = 0; q < 16; ++q)
            hipLaunchKernelGGL(k_greedy_round, dim3(grid_for(B)), dim3(WG), 0, c.stream, B, ap.ptr.get(),
                               ap.col.get(), col.get(), pend.get());
        CS_LAUNCH_CHECK();
        pend.download(hp.data(), hp.size(), c.stream);
        CS_HIP(hipStreamSynchronize(c.stream));
        bool any = false;
        for (int32_t v : hp) any |= (v != 0);
        if (!any) break;
    }
    L.h_colour.resize(B);
    col.download(L.h_colour.data(), B, c.stream);
    CS_HIP(hipStreamSynchronize(c.stream));
    for (int32_t v : L.h_colour)
        if (v < 0) fail(CS_EINVAL, "greedy colouring needs more than 64 colours");
}

// register-blocked M = A~ E for the common block sizes; false: use k_rowprod.
// maxdeg: the most blocks in a block row of A~ (sizes the staging buffer).
bool rowprod_nb(hipStream_t s, int nb, int nl, const int32_t *list, const BPattern &ap, const double *abval,
                const EMat &E, const BPattern &mp, double *mval, int maxdeg) {
    auto go = [&](auto nbc) {
        constexpr int NB = decltype(nbc)::value;
        const int as_n = (int)std::min<int64_t>((int64_t)std::max(maxdeg, 0) * NB * NB, AS_CAP);
        // one wavefront per row while the average row needs at most two of its
        // passes (the first cascade steps: 7 and 25 blocks per row on a 7-point
        // stencil; 128^3 setup 50.1 -> 49.6 ms)
        const int64_t items = (nl > 0 ? mp.nnzb / nl : 0) * (NB % 2 == 0 ? NB / 2 : NB);
        if constexpr (NB <= 8) {
            if (items <= 128) {
                hipLaunchKernelGGL((k_rowprod_nb<NB, 64>), dim3(nl), dim3(64), (size_t)as_n * sizeof(double), s,
                                   list, ap.ptr.get(), ap.col.get(), abval, E.pat.ptr.get(), E.pat.col.get(),
                                   E.val.get(), mp.ptr.get(), mp.col.get(), mval, as_n);
                return true;
            }
        }
        hipLaunchKernelGGL((k_rowprod_nb<NB>), dim3(nl), dim3(WG), (size_t)as_n * sizeof(double), s, list,
                           ap.ptr.get(), ap.col.get(), abval, E.pat.ptr.get(), E.pat.col.get(), E.val.get(),
                           mp.ptr.get(), mp.col.get(), mval, as_n);
        return true;
    };
    switch (nb) {
        case 1: return go(std::integral_constant<int, 1>{});
        case 2: return go(std::integral_constant<int, 2>{});
        case 4: return go(std::integral_constant<int, 4>{});
        case 8: return go(std::integral_constant<int, 8>{});
        case 16: return go(std::integral_constant<int, 16>{});
        default: return false;
    }
}

// Prescaling W = diag(a_kk^{-1/2}), the block pattern of A (when asked for,
// and always for colouring), the colours (multiplicative) and the fit lists:
// the active blocks of one colour at a time (multiplicative), or all active
// blocks at once (additive).
// W of the level: elliptic, or Stokes when the level carries unknown kinds
void compute_prescaling(Ctx &c, Level &L) {
    hipStream_t s = c.stream;
    L.w.alloc(L.n);
    DBuf<int32_t> bad(std::max<int64_t>(L.n, 1));
    if (L.kind.n == (size_t)L.n && L.n > 0) {
        hipLaunchKernelGGL(k_prescale_stokes_v, dim3(grid_for(L.n)), dim3(WG), 0, s, L.a_ptr.get(), L.a_col.get(),
                           L.a_val.get(), L.kind.get(), L.n, L.w.get(), bad.get());
        hipLaunchKernelGGL(k_prescale_stokes_p, dim3(grid_for(L.n)), dim3(WG), 0, s, L.a_ptr.get(), L.a_col.get(),
                           L.a_val.get(), L.kind.get(), L.n, L.stokes_l1, L.w.get(), bad.get());
        CS_LAUNCH_CHECK();
        if (reduce_i32(c, bad.get(), L.n, false))
            fail(CS_EINVAL, "Stokes prescaling: a velocity row without a positive diagonal or a pressure row "
                            "without velocity couplings");
    } else {
        hipLaunchKernelGGL(k_prescale_w, dim3(grid_for(L.n)), dim3(WG), 0, s, L.a_ptr.get(), L.a_col.get(),
                           L.a_val.get(), L.n, L.w.get(), bad.get());
        CS_LAUNCH_CHECK();
        if (reduce_i32(c, bad.get(), L.n, false))
            fail(CS_EINVAL, "elliptic prescaling needs a positive diagonal (declare the unknown kinds of a "
                            "saddle-point level)");
    }
}

struct FitLists {
    std::vector<std::pair<const int32_t *, int>> lists;
    DBuf<int32_t> all_blocks;
};

void prepare_level(Ctx &c, Level &L, const cs_options &o, bool need_ap, BPattern &ap, FitLists &fl) {
    hipStream_t s = c.stream;
    const int B = (int)L.B;
    const int B_act = (int)(L.n_active / L.nb);   // blocks that are smoothed (the rest are solved directly)
    if (L.nb > MAXNB) fail(CS_EINVAL, "block size above 16 is not supported");
    compute_prescaling(c, L);
    if (need_ap || o.mode == CS_MULTIPLICATIVE) block_pattern_of_A(c, L, ap);
    if (o.mode == CS_MULTIPLICATIVE) {
        if (!L.colour_given) greedy_colouring(c, L, ap);
        L.colour.upload(L.h_colour.data(), B, s);
        DBuf<int32_t> bad(B);
        hipLaunchKernelGGL(k_colour_check, dim3(grid_for(B)), dim3(WG), 0, s, B, ap.ptr.get(), ap.col.get(),
                           L.colour.get(), bad.get());
        CS_LAUNCH_CHECK();
        if (reduce_i32(c, bad.get(), B, false))
            fail(CS_ECOLOR, "colouring is not proper: two coupled blocks share a colour");
        if (L.layout_colour != L.h_colour) {   // colours and A unchanged: keep the layout
            build_colour_layout(c, L);
            L.layout_colour = L.h_colour;
        }
        for (int k = 0; k < L.chi; ++k)
            fl.lists.emplace_back(L.cblk.get() + L.cblk_ptr[k], (int)(L.cblk_ptr[k + 1] - L.cblk_ptr[k]));
    } else {
        L.chi = 1;
        fl.all_blocks.alloc(std::max(B_act, 1));
        hipLaunchKernelGGL(k_iota, dim3(grid_for(std::max(B_act, 1))), dim3(WG), 0, s, fl.all_blocks.get(), B_act);
        CS_LAUNCH_CHECK();
        fl.lists.emplace_back(fl.all_blocks.get(), B_act);
    }
}

LatDev lat_dev(const Level &L) {
    return LatDev{L.lat_xyz.get(), L.lat_map.get(), L.lat_lo[0], L.lat_lo[1], L.lat_lo[2],
                  L.lat_ext[0],     L.lat_ext[1],    L.lat_ext[2]};
}

// Translation classes of the smoothed blocks at radius 0 .. depth - 1 into
// L.lat_rep ([depth][B]; other blocks are their own representative) and, per
// radius, the representatives in ascending order.
void lattice_classes(Ctx &c, Level &L, const BPattern &ap, int depth, std::vector<DBuf<int32_t>> &lists,
                     std::vector<int> &sizes) {
    hipStream_t s = c.stream;
    const int B = (int)L.B, nb = (int)L.nb;
    const int Ba = (int)(L.n_active / L.nb);
    const LatDev ld = lat_dev(L);
    DBuf<double> diag(L.n);
    hipLaunchKernelGGL(k_lat_diag, dim3(grid_for(L.n)), dim3(WG), 0, s, L.n, L.a_ptr.get(), L.a_col.get(),
                       L.a_val.get(), diag.get());
    int64_t T = 1;
    while (T < 2 * (int64_t)std::max(Ba, 1) + 1) T <<= 1;
    DBuf<uint64_t> tk(T), key(std::max(Ba, 1));
    DBuf<int32_t> tm(T), flag(std::max(Ba, 1)), off;
    DBuf<int64_t> tot(1);
    L.lat_rep.alloc((size_t)depth * B);
    lists.clear();
    lists.resize(depth);
    sizes.assign(depth, 0);
    for (int r = 0; r < depth; ++r) {
        int32_t *rep = L.lat_rep.get() + (size_t)r * B;
        const int32_t *prev = r ? rep - B : nullptr;
        hipLaunchKernelGGL(k_iota, dim3(grid_for(B)), dim3(WG), 0, s, rep, B);
        CS_LAUNCH_CHECK();
        if (!Ba) continue;
        if (r == 0)
            hipLaunchKernelGGL(k_lat_key0, dim3(grid_for(Ba)), dim3(WG), 0, s, Ba, nb, ap.ptr.get(), ap.col.get(),
                               L.a_ptr.get(), L.a_col.get(), L.a_val.get(), diag.get(), ld, key.get());
        else
            hipLaunchKernelGGL(k_lat_key, dim3(grid_for(Ba)), dim3(WG), 0, s, Ba, ap.ptr.get(), ap.col.get(), ld,
                               prev, key.get());
        hipLaunchKernelGGL(k_lat_clear, dim3(grid_for(T)), dim3(WG), 0, s, T, tk.get(), tm.get());
        hipLaunchKernelGGL(k_lat_insert, dim3(grid_for(Ba)), dim3(WG), 0, s, Ba, key.get(), T, tk.get(), tm.get());
        if (r == 0)
            hipLaunchKernelGGL(k_lat_rep0, dim3(grid_for(Ba)), dim3(WG), 0, s, Ba, nb, ap.ptr.get(), ap.col.get(),
                               L.a_ptr.get(), L.a_col.get(), L.a_val.get(), diag.get(), ld, key.get(), T,
                               tk.get(), tm.get(), rep);
        else
            hipLaunchKernelGGL(k_lat_rep, dim3(grid_for(Ba)), dim3(WG), 0, s, Ba, ap.ptr.get(), ap.col.get(), ld,
                               prev, key.get(), T, tk.get(), tm.get(), rep);
        hipLaunchKernelGGL(k_lat_flag, dim3(grid_for(Ba)), dim3(WG), 0, s, Ba, rep, flag.get());
        CS_LAUNCH_CHECK();
        sizes[r] = (int)scan_counts(c, flag, Ba, off, tot);
        lists[r].alloc(std::max(sizes[r], 1));
        hipLaunchKernelGGL(k_lat_compact, dim3(grid_for(Ba)), dim3(WG), 0, s, Ba, rep, off.get(), lists[r].get());
        CS_LAUNCH_CHECK();
    }
}

void fit_level_overlap_exact(Ctx &c, Level &L, const cs_options &o);

void fit_level(Ctx &c, Level &L, const cs_options &o) {
    if (L.ovl_m) {
        fit_level_overlap_exact(c, L, o);
        return;
    }
    hipStream_t s = c.stream;
    const int B = (int)L.B, nb = (int)L.nb, nb2 = nb * nb;
    const int depth = o.depth;
    BPattern ap;
    FitLists fl;
    prepare_level(c, L, o, true, ap, fl);
    const auto &lists = fl.lists;
    // stencil-repetition cache: fit one block per translation class
    const int B_act = (int)(L.n_active / L.nb);
    const bool lattice = L.lat_dim > 0 && o.mode == CS_ADDITIVE && o.trunc_alpha == 0 && !L.kind.get();
    std::vector<DBuf<int32_t>> lat_lists;
    std::vector<int> lat_sizes;
    L.lat_rep.release();
    L.lat_fitted.assign(depth, B_act);
    DBuf<int32_t> msing, need, lat_acc;   // lat_acc: singular members, translation failures (read at the end)
    if (lattice) {
        lattice_classes(c, L, ap, depth, lat_lists, lat_sizes);
        for (int ell = 0; ell < depth; ++ell) L.lat_fitted[ell] = lat_sizes[ell];
        msing.alloc(B);
        need.alloc(B);
        lat_acc.alloc(2);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(WG), 0, s, lat_acc.get(), (int64_t)2, 0);
    }
    const LatDev ld = lat_dev(L);
    // the prescaled dense blocks of A
    DBuf<double> abval(ap.nnzb * nb2);
    CS_HIP(hipMemsetAsync(abval.get(), 0, abval.bytes(), s));
    hipLaunchKernelGGL(k_scatter_blocks, dim3(grid_for(L.n)), dim3(WG), 0, s, L.a_ptr.get(), L.a_col.get(),
                       L.a_val.get(), L.w.get(), L.n, nb, ap.ptr.get(), ap.col.get(), abval.get());
    CS_LAUNCH_CHECK();
    // E_0 = I
    EMat E;
    E.pat.rows = B;
    E.pat.nnzb = B;
    E.pat.ptr.alloc(B + 1);
    E.pat.col.alloc(B);
    E.val.alloc((size_t)B * nb2);
    hipLaunchKernelGGL(k_identity_E, dim3(grid_for((int64_t)B * nb2)), dim3(WG), 0, s, B, nb, E.pat.ptr.get(),
                       E.pat.col.get(), E.val.get());
    CS_LAUNCH_CHECK();
    auto keep_pattern = [&](const BPattern &p) {
        BPattern q;
        q.rows = p.rows;
        q.nnzb = p.nnzb;
        q.ptr.alloc(p.rows + 1);
        q.col.alloc(std::max<int64_t>(p.nnzb, 1));
        CS_HIP(hipMemcpyAsync(q.ptr.get(), p.ptr.get(), (p.rows + 1) * 4, hipMemcpyDeviceToDevice, s));
        if (p.nnzb) CS_HIP(hipMemcpyAsync(q.col.get(), p.col.get(), p.nnzb * 4, hipMemcpyDeviceToDevice, s));
        L.patterns.push_back(std::move(q));
    };
    L.patterns.clear();
    keep_pattern(E.pat);
    DBuf<double> lamt((size_t)depth * B * nb2);
    CS_HIP(hipMemsetAsync(lamt.get(), 0, lamt.bytes(), s));   // rows of direct segments get no smoother
    DBuf<int32_t> pos(B), sing, cnt, err(B), redo;
    DBuf<int64_t> tot(1);
    const int maxdeg = max_span(c, B, 1, ap.ptr.get());
    int32_t emax = 1;   // longest block row of E (E_0 = I)
    DBuf<int32_t> sing_acc(1);   // singular blocks of the fitted rows, read at the end
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(WG), 0, s, sing_acc.get(), (int64_t)1, 0);
    L.singular = 0;
    const int nsteps = depth * (int)lists.size();
    int step = 0;
    for (int ell = 1; ell <= depth; ++ell) {
        for (size_t kcol = 0; kcol < lists.size(); ++kcol, ++step) {
            const int32_t *dlist = lists[kcol].first;
            int nl = lists[kcol].second;
            const int32_t *lrep = nullptr;   // class representatives at radius ell - 1
            if (lattice) {
                dlist = lat_lists[ell - 1].get();
                nl = lat_sizes[ell - 1];
                lrep = L.lat_rep.get() + (size_t)(ell - 1) * B;
            }
            if (nl == 0) continue;
            hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(B)), dim3(WG), 0, s, pos.get(), (int64_t)B, -1);
            hipLaunchKernelGGL(k_pos_in_list, dim3(grid_for(nl)), dim3(WG), 0, s, dlist, nl, pos.get());
            if (lrep) hipLaunchKernelGGL(k_lat_mark, dim3(grid_for(B)), dim3(WG), 0, s, B, lrep, pos.get());
            hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(B)), dim3(WG), 0, s, err.get(), (int64_t)B, 0);
            // symbolic: pattern(M_i) for the list rows
            cnt.alloc(nl);
            BPattern mp;
            mp.rows = nl;
            const int64_t bound = maxdeg <= 64 ? (int64_t)maxdeg * emax : INT64_MAX;
            launch_union<SRC_E, false>(s, bound, dlist, nl, nb, ap.ptr.get(), ap.col.get(), E.pat.ptr.get(),
                                       E.pat.col.get(), cnt.get(), nullptr, nullptr, err.get());
            CS_LAUNCH_CHECK();
            int32_t overflow = 0;
            mp.nnzb = scan_counts_ex(c, cnt, nl, mp.ptr, tot, nullptr, err.get(), nl, &overflow);
            if (overflow) fail(CS_EINVAL, "fill of a residual row exceeds the per-row capacity of the symbolic kernels");
            mp.col.alloc(mp.nnzb);
            launch_union<SRC_E, true>(s, bound, dlist, nl, nb, ap.ptr.get(), ap.col.get(), E.pat.ptr.get(),
                                      E.pat.col.get(), nullptr, mp.ptr.get(), mp.col.get(), err.get());
            CS_LAUNCH_CHECK();
            // numeric: M, normal equations, Lambda~
            DBuf<double> mval((size_t)mp.nnzb * nb2);
            if (nb == 1)
                hipLaunchKernelGGL(k_rowprod_point, dim3((unsigned)ceil_div(nl, WG / 64)), dim3(WG), 0, s, nl,
                                   dlist, ap.ptr.get(), ap.col.get(), abval.get(), E.pat.ptr.get(),
                                   E.pat.col.get(), E.val.get(), mp.ptr.get(), mp.col.get(), mval.get());
            else if (!rowprod_nb(s, nb, nl, dlist, ap, abval.get(), E, mp, mval.get(), maxdeg))
                hipLaunchKernelGGL(k_rowprod, dim3(nl), dim3(WG), 0, s, dlist, nb, ap.ptr.get(), ap.col.get(),
                                   abval.get(), E.pat.ptr.get(), E.pat.col.get(), E.val.get(), mp.ptr.get(),
                                   mp.col.get(), mval.get());
            CS_LAUNCH_CHECK();
            sing.alloc(nl);
            double *lam_l = lamt.get() + (size_t)(ell - 1) * B * nb2;
            if (nb == 1)
                hipLaunchKernelGGL(k_gram_point, dim3((unsigned)ceil_div(nl, WG / 64)), dim3(WG), 0, s, nl,
                                   dlist, mp.ptr.get(), mp.col.get(), mval.get(), E.pat.ptr.get(),
                                   E.pat.col.get(), E.val.get(), lam_l, sing.get(), o.ridge);
            else {
                auto go = [&](auto nbc) {
                    constexpr int NBT = decltype(nbc)::value;
                    hipLaunchKernelGGL((k_gram_solve<NBT>), dim3(nl), dim3(WG), 0, s, nl, dlist, nb, mp.ptr.get(),
                                       mp.col.get(), mval.get(), E.pat.ptr.get(), E.pat.col.get(), E.val.get(),
                                       lam_l, sing.get(), o.ridge, (const int32_t *)nullptr);
                };
                switch (nb) {
                    case 2: go(std::integral_constant<int, 2>{}); break;
                    case 4: go(std::integral_constant<int, 4>{}); break;
                    case 8:
                        // matrix cores, then the rows they flag through the minimum-norm path
                        if (redo.n < (size_t)nl + 1) redo.alloc((size_t)nl + 1);   // grow only: a free syncs
                        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(WG), 0, s, redo.get(), (int64_t)1, 0);
                        hipLaunchKernelGGL(k_gram_mfma8, dim3((unsigned)ceil_div(nl, 8)), dim3(WG), 0, s, nl, dlist,
                                           mp.ptr.get(), mp.col.get(), mval.get(), E.pat.ptr.get(),
                                           E.pat.col.get(), E.val.get(), lam_l, sing.get(), redo.get(), o.ridge);
                        hipLaunchKernelGGL((k_gram_solve<8>), dim3(256), dim3(WG), 0, s, nl, dlist, nb, mp.ptr.get(),
                                           mp.col.get(), mval.get(), E.pat.ptr.get(), E.pat.col.get(), E.val.get(),
                                           lam_l, sing.get(), o.ridge, (const int32_t *)redo.get());
                        break;
                    case 16:
                        hipLaunchKernelGGL(k_gram_mfma, dim3(nl), dim3(WG), 0, s, dlist, mp.ptr.get(),
                                           mp.col.get(), mval.get(), E.pat.ptr.get(), E.pat.col.get(),
                                           E.val.get(), lam_l, sing.get(), o.ridge);
                        break;
                    default: go(std::integral_constant<int, 0>{}); break;
                }
            }
            hipLaunchKernelGGL(k_reduce_i32<true>, dim3(std::min<unsigned>(grid_for(nl), 4096)), dim3(WG), 0, s,
                               (int64_t)nl, sing.get(), sing_acc.get());
            CS_LAUNCH_CHECK();
            if (lrep) {
                hipLaunchKernelGGL(k_lat_copy_lam, dim3(grid_for((int64_t)B * nb2)), dim3(WG), 0, s, B, nb2, lrep,
                                   pos.get(), sing.get(), lam_l, msing.get());
                hipLaunchKernelGGL(k_reduce_i32<true>, dim3(std::min<unsigned>(grid_for(B), 4096)), dim3(WG), 0, s,
                                   (int64_t)B, msing.get(), lat_acc.get());
                CS_LAUNCH_CHECK();
            }
            if (step + 1 == nsteps) break;   // the last residual is never needed
            // E update on pattern(M) for list rows, copy for others
            {
                DBuf<int32_t> ncnt(B);
                hipLaunchKernelGGL(k_ecount, dim3(grid_for(B)), dim3(WG), 0, s, B, pos.get(), lrep, mp.ptr.get(),
                                   E.pat.ptr.get(), ncnt.get());
                CS_LAUNCH_CHECK();
                EMat N;
                N.pat.rows = B;
                N.pat.nnzb = scan_counts_ex(c, ncnt, B, N.pat.ptr, tot, &emax, nullptr, 0, nullptr);
                N.pat.col.alloc(N.pat.nnzb);
                N.val.alloc((size_t)N.pat.nnzb * nb2);
                launch_eupdate(s, B, nb, pos.get(), mp.ptr.get(), mp.col.get(), mval.get(), E.pat.ptr.get(),
                               E.pat.col.get(), E.val.get(), lam_l, N.pat.ptr.get(), N.pat.col.get(), N.val.get());
                CS_LAUNCH_CHECK();
                if (lrep) {
                    // rows read by step ell + 1: its list (the classes at radius ell) and their neighbours
                    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(B)), dim3(WG), 0, s, need.get(), (int64_t)B, 0);
                    hipLaunchKernelGGL(k_lat_need, dim3(grid_for(lat_sizes[ell])), dim3(WG), 0, s, lat_sizes[ell],
                                       lat_lists[ell].get(), ap.ptr.get(), ap.col.get(), need.get());
                    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(B)), dim3(WG), 0, s, err.get(), (int64_t)B, 0);
                    hipLaunchKernelGGL(k_lat_etranslate, dim3(B), dim3(WG), 0, s, B, nb, pos.get(), lrep, ld,
                                       need.get(), N.pat.ptr.get(), N.pat.col.get(), N.val.get(), err.get());
                    hipLaunchKernelGGL(k_reduce_i32<false>, dim3(std::min<unsigned>(grid_for(B), 4096)), dim3(WG),
                                       0, s, (int64_t)B, err.get(), lat_acc.get() + 1);
                    CS_LAUNCH_CHECK();
                }
                mval.release();
                if (o.trunc_alpha > 0) {
                    DBuf<int32_t> tcnt(B);
                    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(B)), dim3(WG), 0, s, err.get(), (int64_t)B, 0);
                    hipLaunchKernelGGL((k_truncate<false>), dim3(B), dim3(WG), 0, s, B, nb, o.trunc_alpha, pos.get(),
                                       N.pat.ptr.get(), N.pat.col.get(), N.val.get(), tcnt.get(), nullptr, nullptr,
                                       nullptr, err.get());
                    CS_LAUNCH_CHECK();
                    int32_t tover = 0;
                    EMat T;
                    T.pat.rows = B;
                    T.pat.nnzb = scan_counts_ex(c, tcnt, B, T.pat.ptr, tot, &emax, err.get(), B, &tover);
                    if (tover)
                        fail(CS_EINVAL, "truncated residual row exceeds the per-row capacity of the symbolic kernels");
                    T.pat.col.alloc(T.pat.nnzb);
                    T.val.alloc((size_t)T.pat.nnzb * nb2);
                    hipLaunchKernelGGL((k_truncate<true>), dim3(B), dim3(WG), 0, s, B, nb, o.trunc_alpha, pos.get(),
                                       N.pat.ptr.get(), N.pat.col.get(), N.val.get(), nullptr, T.pat.ptr.get(),
                                       T.pat.col.get(), T.val.get(), err.get());
                    CS_LAUNCH_CHECK();
                    N = std::move(T);
                }
                E = std::move(N);
                keep_pattern(E.pat);
            }
        }
    }
    {
        int32_t acc[2] = {0, 0}, sg = 0;
        sing_acc.download(&sg, 1, s);
        if (lattice) lat_acc.download(acc, 2, s);
        CS_HIP(hipStreamSynchronize(s));
        if (acc[1])
            fail(CS_EINVAL, "a residual row of a lattice class could not be translated (row above " +
                                std::to_string(LAT_ROW_CAP) + " blocks, or a neighbour off the lattice)");
        L.singular = sg + acc[0];
    }
    // unscale into the FP64 master
    L.depth = depth;
    L.lam64.alloc((size_t)depth * B * nb2);
    for (int ell = 0; ell < depth; ++ell)
        hipLaunchKernelGGL(k_unscale, dim3(grid_for((int64_t)B * nb2)), dim3(WG), 0, s, (int64_t)B, nb, L.w.get(),
                           lamt.get() + (size_t)ell * B * nb2, L.lam64.get() + (size_t)ell * B * nb2);
    CS_LAUNCH_CHECK();
    CS_HIP(hipStreamSynchronize(s));
}

// Exact fit of a level with overlapping blocks (Sec. 3.6.2): scalar residual
// E (CSR over nodes), per cascade level M = A~ E on every node (symbolic union
// and the point row product), the blockwise normal equations over the slots,
// and E_new = diag(theta)^{-1} Theta^T (Theta E - Lambda~ Theta M) row by row.
void fit_level_overlap_exact(Ctx &c, Level &L, const cs_options &o) {
    L.lat_fitted.clear();
    L.lat_rep.release();
    hipStream_t s = c.stream;
    const int depth = o.depth, m = L.ovl_m;
    const int64_t n = L.n, nblk = L.ovl_nblk, m2 = (int64_t)m * m;
    compute_prescaling(c, L);
    L.patterns.clear();
    // A~ on the scalar pattern of A
    BPattern ap;
    ap.rows = n;
    ap.nnzb = L.nnz;
    ap.ptr.alloc(n + 1);
    ap.col.alloc(std::max<int64_t>(L.nnz, 1));
    CS_HIP(hipMemcpyAsync(ap.ptr.get(), L.a_ptr.get(), (n + 1) * 4, hipMemcpyDeviceToDevice, s));
    CS_HIP(hipMemcpyAsync(ap.col.get(), L.a_col.get(), L.nnz * 4, hipMemcpyDeviceToDevice, s));
    DBuf<double> aval(std::max<int64_t>(L.nnz, 1));
    hipLaunchKernelGGL(k_prescaled_csr, dim3(grid_for(n)), dim3(WG), 0, s, n, L.a_ptr.get(), L.a_col.get(),
                       L.a_val.get(), L.w.get(), aval.get());
    // E_0 = I
    EMat E;
    E.pat.rows = n;
    E.pat.nnzb = n;
    E.pat.ptr.alloc(n + 1);
    E.pat.col.alloc(n);
    E.val.alloc(n);
    hipLaunchKernelGGL(k_identity_E, dim3(grid_for(n)), dim3(WG), 0, s, (int)n, 1, E.pat.ptr.get(), E.pat.col.get(),
                       E.val.get());
    CS_LAUNCH_CHECK();
    DBuf<int32_t> list(n), cnt(n), err(n), sing(nblk);
    DBuf<int64_t> tot(1);
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(WG), 0, s, list.get(), (int)n);
    DBuf<double> lamt((size_t)depth * nblk * m2), gh((size_t)nblk * 2 * m2);
    const int maxdeg = max_span(c, n, 1, ap.ptr.get());
    const dim3 gw((unsigned)ceil_div(n, WG / 64)), gb((unsigned)ceil_div(nblk, WG / 64));
    L.singular = 0;
    for (int ell = 1; ell <= depth; ++ell) {
        // symbolic and numeric M = A~ E on every node
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(WG), 0, s, err.get(), n, 0);
        BPattern mp;
        mp.rows = n;
        const int64_t bound = maxdeg <= 64 ? (int64_t)maxdeg * max_span(c, n, 1, E.pat.ptr.get()) : INT64_MAX;
        launch_union<SRC_E, false>(s, bound, list.get(), (int)n, 1, ap.ptr.get(), ap.col.get(), E.pat.ptr.get(),
                                   E.pat.col.get(), cnt.get(), nullptr, nullptr, err.get());
        CS_LAUNCH_CHECK();
        check_flags(c, err, n, "fill of a residual row");
        mp.nnzb = scan_counts(c, cnt, n, mp.ptr, tot);
        mp.col.alloc(std::max<int64_t>(mp.nnzb, 1));
        launch_union<SRC_E, true>(s, bound, list.get(), (int)n, 1, ap.ptr.get(), ap.col.get(), E.pat.ptr.get(),
                                  E.pat.col.get(), nullptr, mp.ptr.get(), mp.col.get(), err.get());
        DBuf<double> mval(std::max<int64_t>(mp.nnzb, 1));
        hipLaunchKernelGGL(k_rowprod_point, gw, dim3(WG), 0, s, (int)n, list.get(), ap.ptr.get(), ap.col.get(),
                           aval.get(), E.pat.ptr.get(), E.pat.col.get(), E.val.get(), mp.ptr.get(), mp.col.get(),
                           mval.get());
        // normal equations per overlapping block
        double *lam_l = lamt.get() + (size_t)(ell - 1) * nblk * m2;
        hipLaunchKernelGGL(k_ovl_gram_sparse, gb, dim3(WG), 0, s, nblk, m, L.ovl_nodes.get(), mp.ptr.get(),
                           mp.col.get(), mval.get(), E.pat.ptr.get(), E.pat.col.get(), E.val.get(), gh.get());
        hipLaunchKernelGGL(k_sk_solve, dim3((unsigned)nblk), dim3(WG), 0, s, list.get(), m, (const double *)gh.get(),
                           lam_l, sing.get(), 0.0);
        CS_LAUNCH_CHECK();
        L.singular += reduce_i32(c, sing.get(), nblk, true);
        if (ell == depth) break;
        // new residual rows
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(WG), 0, s, err.get(), n, 0);
        hipLaunchKernelGGL(k_ovl_union<false>, dim3((unsigned)n), dim3(WG), 0, s, n, m, L.ovl_nodes.get(),
                           L.ovl_inv_ptr.get(), L.ovl_inv_idx.get(), E.pat.ptr.get(), E.pat.col.get(), mp.ptr.get(),
                           mp.col.get(), cnt.get(), nullptr, nullptr, err.get());
        CS_LAUNCH_CHECK();
        check_flags(c, err, n, "fill of an overlapping residual row");
        EMat N;
        N.pat.rows = n;
        N.pat.nnzb = scan_counts(c, cnt, n, N.pat.ptr, tot);
        N.pat.col.alloc(std::max<int64_t>(N.pat.nnzb, 1));
        N.val.alloc(std::max<int64_t>(N.pat.nnzb, 1));
        hipLaunchKernelGGL(k_ovl_union<true>, dim3((unsigned)n), dim3(WG), 0, s, n, m, L.ovl_nodes.get(),
                           L.ovl_inv_ptr.get(), L.ovl_inv_idx.get(), E.pat.ptr.get(), E.pat.col.get(), mp.ptr.get(),
                           mp.col.get(), nullptr, N.pat.ptr.get(), N.pat.col.get(), err.get());
        hipLaunchKernelGGL(k_ovl_eupdate, gw, dim3(WG), 0, s, n, m, L.ovl_nodes.get(), L.ovl_inv_ptr.get(),
                           L.ovl_inv_idx.get(), L.ovl_rtheta.get(), (const double *)lam_l, E.pat.ptr.get(),
                           E.pat.col.get(), E.val.get(), mp.ptr.get(), mp.col.get(), mval.get(), N.pat.ptr.get(),
                           N.pat.col.get(), N.val.get());
        CS_LAUNCH_CHECK();
        E = std::move(N);
    }
    L.depth = depth;
    L.lam64.alloc((size_t)depth * nblk * m2);
    for (int ell = 0; ell < depth; ++ell)
        hipLaunchKernelGGL(k_ovl_unscale, dim3(grid_for(nblk * m2)), dim3(WG), 0, s, nblk, m, L.ovl_nodes.get(),
                           L.w.get(), lamt.get() + (size_t)ell * nblk * m2, L.lam64.get() + (size_t)ell * nblk * m2);
    CS_LAUNCH_CHECK();
    CS_HIP(hipStreamSynchronize(s));
}

// Sketched fit of a level with overlapping blocks (Sec. 3.6.2 with the sketch
// of Sec. 4): per cascade level M = A~ T, the blockwise normal equations over
// the replicated slots, then T <- diag(theta)^{-1} Theta^T (Theta T - Lambda~ Theta M),
// i.e. T_k -= (1/theta_k) sum over the slots of k of (Lambda~ M)_slot.
void fit_level_overlap_sketched(Ctx &c, Level &L, const cs_options &o, const double *S, int sk) {
    hipStream_t s = c.stream;
    const int depth = o.depth, m = L.ovl_m;
    const int64_t nblk = L.ovl_nblk, m2 = (int64_t)m * m;
    compute_prescaling(c, L);
    L.patterns.clear();
    const size_t nT = (size_t)L.n * sk;
    DBuf<double> T(std::max<size_t>(nT, 1)), M(std::max<size_t>(nT, 1));
    CS_HIP(hipMemcpyAsync(T.get(), S, nT * sizeof(double), hipMemcpyDeviceToDevice, s));
    DBuf<double> lamt((size_t)depth * nblk * m2), gh((size_t)nblk * 2 * m2), Y((size_t)nblk * m * sk);
    DBuf<int32_t> list(nblk), sing(nblk);
    hipLaunchKernelGGL(k_iota, dim3(grid_for(nblk)), dim3(WG), 0, s, list.get(), (int)nblk);
    CS_LAUNCH_CHECK();
    const dim3 gr((unsigned)ceil_div(L.n, WG / 64)), gb((unsigned)ceil_div(nblk, WG / 64));
    L.singular = 0;
    for (int ell = 1; ell <= depth; ++ell) {
        double *lam_l = lamt.get() + (size_t)(ell - 1) * nblk * m2;
        hipLaunchKernelGGL(k_sk_rows, gr, dim3(WG), 0, s, L.n, L.a_ptr.get(), L.a_col.get(), L.a_val.get(),
                           L.w.get(), sk, (const double *)T.get(), M.get());
        auto go = [&](auto mbc) {
            constexpr int MB = decltype(mbc)::value;
            hipLaunchKernelGGL(k_ovl_gram<MB>, gb, dim3(WG), 0, s, nblk, m, L.ovl_nodes.get(), sk,
                               (const double *)M.get(), (const double *)T.get(), gh.get());
            hipLaunchKernelGGL(k_sk_solve, dim3((unsigned)nblk), dim3(WG), 0, s, list.get(), m,
                               (const double *)gh.get(), lam_l, sing.get(), 0.0);
            if (ell < depth) {
                hipLaunchKernelGGL(k_ovl_y<MB>, gb, dim3(WG), 0, s, nblk, m, L.ovl_nodes.get(), sk,
                                   (const double *)lam_l, (const double *)M.get(), Y.get());
                hipLaunchKernelGGL(k_ovl_fuse_T, gr, dim3(WG), 0, s, L.n, L.ovl_inv_ptr.get(), L.ovl_inv_idx.get(),
                                   L.ovl_rtheta.get(), sk, (const double *)Y.get(), T.get());
            }
        };
        if (m <= 4) go(std::integral_constant<int, 4>{});
        else if (m <= 8) go(std::integral_constant<int, 8>{});
        else go(std::integral_constant<int, 16>{});
        CS_LAUNCH_CHECK();
        L.singular += reduce_i32(c, sing.get(), nblk, true);
    }
    L.depth = depth;
    L.lam64.alloc((size_t)depth * nblk * m2);
    for (int ell = 0; ell < depth; ++ell)
        hipLaunchKernelGGL(k_ovl_unscale, dim3(grid_for(nblk * m2)), dim3(WG), 0, s, nblk, m, L.ovl_nodes.get(),
                           L.w.get(), lamt.get() + (size_t)ell * nblk * m2, L.lam64.get() + (size_t)ell * nblk * m2);
    CS_LAUNCH_CHECK();
    CS_HIP(hipStreamSynchronize(s));
}

// Sketched fit of one level (Sec. 4): T_0 = S (N x s, device, row-major),
// then for every cascade level and fit list: M = A~ T on the list blocks, the
// normal equations of min ||T_i - Lambda~_i M_i||_F, T_i <- T_i - Lambda~_i M_i.
void fit_level_sketched(Ctx &c, Level &L, const cs_options &o, const double *S, int sk) {
    if (L.ovl_m) {
        fit_level_overlap_sketched(c, L, o, S, sk);
        return;
    }
    hipStream_t s = c.stream;
    const int B = (int)L.B, nb = (int)L.nb, nb2 = nb * nb;
    const int depth = o.depth;
    BPattern ap;
    FitLists fl;
    prepare_level(c, L, o, false, ap, fl);
    L.patterns.clear();   // no residual patterns: the sketch is dense
    const size_t nT = (size_t)L.n * sk;
    // point blocks update T inside the fitting kernel: additive steps write a
    // second buffer (every block reads its neighbours' old rows), colour steps
    // update in place (a proper colouring couples no two blocks of one colour)
    const bool pingpong = nb == 1 && o.mode == CS_ADDITIVE;
    DBuf<double> T0(std::max<size_t>(nT, 1)), T1(pingpong ? std::max<size_t>(nT, 1) : 1);
    CS_HIP(hipMemcpyAsync(T0.get(), S, nT * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (pingpong) CS_HIP(hipMemcpyAsync(T1.get(), S, nT * sizeof(double), hipMemcpyDeviceToDevice, s));
    double *Tin = T0.get(), *Tout = pingpong ? T1.get() : T0.get();
    DBuf<double> lamt((size_t)depth * B * nb2);
    CS_HIP(hipMemsetAsync(lamt.get(), 0, lamt.bytes(), s));   // rows of direct segments get no smoother
    int maxl = 1;
    for (const auto &pr : fl.lists) maxl = std::max(maxl, pr.second);
    DBuf<int32_t> sing(maxl);
    DBuf<double> Mb(nb > 1 ? (size_t)maxl * nb * sk : 1), gh(nb > 1 ? (size_t)maxl * 2 * nb2 : 1);
    L.singular = 0;
    for (int ell = 1; ell <= depth; ++ell) {
        double *lam_l = lamt.get() + (size_t)(ell - 1) * B * nb2;
        for (const auto &pr : fl.lists) {
            const int32_t *list = pr.first;
            const int nl = pr.second;
            if (nl == 0) continue;
            const dim3 gw((unsigned)ceil_div(nl, WG / 64));
            if (nb == 1) {
                hipLaunchKernelGGL(k_sk_point, gw, dim3(WG), 0, s, nl, list, L.a_ptr.get(), L.a_col.get(),
                                   L.a_val.get(), L.w.get(), sk, Tin, Tout, lam_l, sing.get());
                CS_LAUNCH_CHECK();
                if (pingpong) std::swap(Tin, Tout);
            } else {
                auto go = [&](auto nbc) {
                    constexpr int NB = decltype(nbc)::value;
                    hipLaunchKernelGGL(k_sk_gram<NB>, gw, dim3(WG), 0, s, nl, list, L.a_ptr.get(), L.a_col.get(),
                                       L.a_val.get(), L.w.get(), sk, (const double *)Tin, Mb.get(), gh.get());
                    hipLaunchKernelGGL(k_sk_solve, dim3((unsigned)nl), dim3(WG), 0, s, list, nb,
                                       (const double *)gh.get(), lam_l, sing.get(), 0.0);
                    hipLaunchKernelGGL(k_sk_update<NB>, gw, dim3(WG), 0, s, nl, list, sk, (const double *)lam_l,
                                       (const double *)Mb.get(), Tin);
                };
                switch (nb) {
                    case 2: go(std::integral_constant<int, 2>{}); break;
                    case 4: go(std::integral_constant<int, 4>{}); break;
                    case 8: go(std::integral_constant<int, 8>{}); break;
                    case 16: go(std::integral_constant<int, 16>{}); break;
                    default: fail(CS_EINVAL, "the sketched setup supports block sizes 1, 2, 4, 8 and 16");
                }
                CS_LAUNCH_CHECK();
            }
            L.singular += reduce_i32(c, sing.get(), nl, true);
        }
    }
    L.depth = depth;
    L.lam64.alloc((size_t)depth * B * nb2);
    for (int ell = 0; ell < depth; ++ell)
        hipLaunchKernelGGL(k_unscale, dim3(grid_for((int64_t)B * nb2)), dim3(WG), 0, s, (int64_t)B, nb, L.w.get(),
                           lamt.get() + (size_t)ell * B * nb2, L.lam64.get() + (size_t)ell * B * nb2);
    CS_LAUNCH_CHECK();
    CS_HIP(hipStreamSynchronize(s));
}

}  // namespace

void factor_direct(Ctx &c, Level &L) {
    const int nseg = (int)L.dseg.size() - 1;
    if (nseg <= 0) return;
    // dense copies of the segment diagonal blocks of A, concatenated
    std::vector<double> dense(L.dinv.n, 0.0);
    size_t off = 0;
    for (int q = 0; q < nseg; ++q) {
        const int64_t r0 = L.dseg[q], m = L.dseg[q + 1] - r0;
        for (int64_t r = r0; r < r0 + m; ++r)
            for (int64_t e = L.h_ptr[r]; e < L.h_ptr[r + 1]; ++e)
                dense[off + (size_t)(r - r0) * m + (L.h_col[e] - r0)] += L.h_val[e];
        off += (size_t)m * m;
    }
    // pack the segments largest first: step k then works on the prefix of
    // segments larger than k only
    std::vector<int> ord(nseg);
    for (int q = 0; q < nseg; ++q) ord[q] = q;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
        return L.dseg[x + 1] - L.dseg[x] > L.dseg[y + 1] - L.dseg[y];
    });
    std::vector<int64_t> src_off(nseg + 1, 0), soff(nseg + 1, 0), dst_off(nseg);
    std::vector<int32_t> msz(nseg);
    for (int q = 0; q < nseg; ++q) {
        const int64_t m = L.dseg[q + 1] - L.dseg[q];
        src_off[q + 1] = src_off[q] + m * m;
    }
    std::vector<double> packed(dense.size());
    for (int t = 0; t < nseg; ++t) {
        const int q = ord[t];
        const int64_t m = L.dseg[q + 1] - L.dseg[q];
        msz[t] = (int32_t)m;
        dst_off[t] = src_off[q];
        soff[t + 1] = soff[t] + m * m;
        std::copy(dense.begin() + src_off[q], dense.begin() + src_off[q + 1], packed.begin() + soff[t]);
    }
    const int64_t tot = (int64_t)L.dinv.n;
    DBuf<double> a(tot), b(tot);
    DBuf<int64_t> soff_d, dst_d;
    DBuf<int32_t> msz_d;
    a.upload(packed.data(), packed.size(), c.stream);
    soff_d.upload(soff.data(), soff.size(), c.stream);
    dst_d.upload(dst_off.data(), dst_off.size(), c.stream);
    msz_d.upload(msz.data(), msz.size(), c.stream);
    // step k reads buffer (k even ? a : b) and writes the other one
    int nact = nseg;
    for (int k = 0; k < L.dseg_max; ++k) {
        while (nact > 0 && msz[nact - 1] <= k) --nact;
        const int64_t n_el = soff[nact];
        const double *in = (k & 1) ? b.get() : a.get();
        double *out = (k & 1) ? a.get() : b.get();
        hipLaunchKernelGGL(k_gauss_jordan_seg, dim3(grid_for(n_el)), dim3(WG), 0, c.stream, in, out, nact,
                           soff_d.get(), msz_d.get(), k);
    }
    hipLaunchKernelGGL(k_gauss_jordan_collect, dim3(grid_for(tot)), dim3(WG), 0, c.stream, tot, nseg, soff_d.get(),
                       msz_d.get(), dst_d.get(), a.get(), b.get(), L.dinv.get());
    CS_LAUNCH_CHECK();
    CS_HIP(hipStreamSynchronize(c.stream));
}

void build_working_copies(Ctx &c) {
    c.gen++;   // buffers change: captured graphs are stale
    for (size_t l = 0; l + 1 < c.lv.size(); ++l) {
        Level &L = c.lv[l];
        const int64_t nbk = lam_count(L), bsz = lam_size(L);
        const int64_t tot = (int64_t)L.depth * nbk * bsz * bsz;
        L.lam64T.alloc(tot);
        hipLaunchKernelGGL(k_transpose_blocks64, dim3(grid_for(tot)), dim3(WG), 0, c.stream, (int64_t)L.depth * nbk,
                           (int)bsz, L.lam64.get(), L.lam64T.get());
        L.lam32.alloc(tot);
        L.lam32T.alloc(tot);
        hipLaunchKernelGGL(k_cast32, dim3(grid_for(tot)), dim3(WG), 0, c.stream, tot, L.lam64.get(), L.lam32.get());
        hipLaunchKernelGGL(k_cast32, dim3(grid_for(tot)), dim3(WG), 0, c.stream, tot, L.lam64T.get(), L.lam32T.get());
        CS_LAUNCH_CHECK();
        if (!L.ovl_m) build_bf16_smoother(c, L);
    }
    CS_HIP(hipStreamSynchronize(c.stream));
}

// Every cascade level of L is omega A_ii^{-1} (cs_options.source =
// CS_SRC_JACOBI): no fit; the prescaling, colouring and layouts as for a fit.
void jacobi_level(Ctx &c, Level &L, const cs_options &o) {
    hipStream_t s = c.stream;
    BPattern ap;
    FitLists fl;
    prepare_level(c, L, o, false, ap, fl);
    L.patterns.clear();
    L.lat_fitted.clear();
    L.lat_rep.release();
    L.singular = 0;
    L.depth = o.depth;
    const int64_t B = L.B, B_act = L.n_active / L.nb;
    L.lam64.alloc((size_t)o.depth * B * L.nb * L.nb);
    DBuf<int32_t> bad(std::max<int64_t>(B, 1));
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(std::max<int64_t>(B, 1))), dim3(WG), 0, s, bad.get(),
                       std::max<int64_t>(B, 1), 0);
    hipLaunchKernelGGL(k_block_jacobi, dim3((unsigned)((B + WG / 64 - 1) / (WG / 64))), dim3(WG), 0, s, B, B_act,
                       (int)L.nb, o.depth, o.jacobi_omega, L.a_ptr.get(), L.a_col.get(), L.a_val.get(),
                       L.lam64.get(), bad.get());
    CS_LAUNCH_CHECK();
    if (reduce_i32(c, bad.get(), std::max<int64_t>(B, 1), false))
        fail(CS_ESINGULAR, "block Jacobi: a diagonal block of A is singular");
}

void run_setup(Ctx &c, const cs_options &o) {
    CS_HIP(hipEventRecord(c.ev0, c.stream));
    c.singular = 0;
    for (size_t l = 0; l + 1 < c.lv.size(); ++l) {
        if (o.source == CS_SRC_JACOBI) jacobi_level(c, c.lv[l], o);
        else fit_level(c, c.lv[l], o);
        c.singular += c.lv[l].singular;
    }
    for (Level &L : c.lv) factor_direct(c, L);
    build_working_copies(c);
    CS_HIP(hipEventRecord(c.ev1, c.stream));
    CS_HIP(hipEventSynchronize(c.ev1));
    float ms = 0;
    CS_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
    c.setup_ms = ms;
}

void run_setup_sketched(Ctx &c, const cs_options &o, int sk, const double *S) {
    CS_HIP(hipEventRecord(c.ev0, c.stream));
    c.singular = 0;
    for (Level &L : c.lv) {   // no exact block fit: no class statistics
        L.lat_fitted.clear();
        L.lat_rep.release();
    }
    size_t off = 0;
    for (size_t l = 0; l + 1 < c.lv.size(); ++l) {
        fit_level_sketched(c, c.lv[l], o, S + off, sk);
        off += (size_t)c.lv[l].n * sk;
        c.singular += c.lv[l].singular;
    }
    for (Level &L : c.lv) factor_direct(c, L);
    build_working_copies(c);
    CS_HIP(hipEventRecord(c.ev1, c.stream));
    CS_HIP(hipEventSynchronize(c.ev1));
    float ms = 0;
    CS_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
    c.setup_ms = ms;
}

namespace {
void level_prescaling(Ctx &c, Level &L) {
    if (L.w.n == (size_t)L.n) return;
    compute_prescaling(c, L);
}
}  // namespace

void prescaled_blocks(Ctx &c, Level &L, float *out) {
    level_prescaling(c, L);
    const int64_t tot = (int64_t)L.depth * L.B * L.nb * L.nb;
    hipLaunchKernelGGL(k_prescaled_export, dim3(grid_for(tot)), dim3(WG), 0, c.stream, L.B, (int)L.nb, L.depth,
                       L.w.get(), L.lam64.get(), out);
    CS_LAUNCH_CHECK();
    CS_HIP(hipStreamSynchronize(c.stream));
}

void run_setup_learned(Ctx &c, const cs_options &o, const float *lam_t) {
    // lam_t is produced on c.stream before this call; timing covers it
    Level &L0 = c.lv[0];
    const int nb2 = (int)(L0.nb * L0.nb);
    L0.w.release();
    level_prescaling(c, L0);
    L0.depth = o.depth;
    L0.lam64.alloc((size_t)o.depth * L0.B * nb2);
    const int64_t tot = (int64_t)o.depth * L0.B * nb2;
    hipLaunchKernelGGL(k_unscale_learned, dim3(grid_for(tot)), dim3(WG), 0, c.stream, L0.B, (int)L0.nb, o.depth,
                       L0.w.get(), lam_t, L0.lam64.get());
    CS_LAUNCH_CHECK();
    L0.patterns.clear();
    L0.singular = 0;
    L0.chi = 1;
    L0.lat_fitted.clear();
    L0.lat_rep.release();
    c.singular = 0;
    for (size_t l = 1; l + 1 < c.lv.size(); ++l) {
        fit_level(c, c.lv[l], o);
        c.singular += c.lv[l].singular;
    }
    for (Level &L : c.lv) factor_direct(c, L);
    build_working_copies(c);
}

}  // namespace cs
