// Internal declarations of the cascading-smoother multigrid library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cascade.h"

namespace cs {

struct Error {
    cs_status st;
    std::string msg;
};

[[noreturn]] inline void fail(cs_status st, const std::string &msg) { throw Error{st, msg}; }

#define CS_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            ::cs::fail(CS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

#define CS_LAUNCH_CHECK() CS_HIP(hipGetLastError())

// Map the hardware workgroup id (of G) to a logical index so that each of the
// 8 XCDs (which receive workgroups round-robin) works through one contiguous
// range: neighbouring rows, which read the same gathered data, then run on the
// same XCD and share its L2.  A bijection of [0, G).
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t G) {
    const int64_t xcd = bid & 7, idx = bid >> 3;
    const int64_t per = G >> 3, rem = G & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// Device memory cache (pool.hip): blocks are reused across allocations; a
// freed block is released to the cache after a device synchronisation.
void *pool_alloc(size_t bytes);   // throws CS_ENOMEM
void pool_free(void *p);
void pool_user(int delta);        // contexts alive; the cache is emptied when none are

// Owning device buffer.
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        p = static_cast<T *>(pool_alloc(count * sizeof(T)));
        n = count;
    }
    void release() {
        if (p) pool_free(p);
        p = nullptr;
        n = 0;
    }
    T *get() const { return p; }
    size_t bytes() const { return n * sizeof(T); }
    void upload(const T *h, size_t count, hipStream_t s) {
        if (count > n) alloc(count);
        if (count) CS_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void download(T *h, size_t count, hipStream_t s) const {
        if (count) CS_HIP(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    }
};

// Sliced ELLPACK (slice height 64 = one wavefront) of a scalar sparse matrix,
// over a list of rows (rows == nullptr: rows 0..nrows-1 in order).  Entry k of
// lane l in slice s sits at slice_ptr[s] + k*64 + l; padding entries point at
// the row itself with value 0.
struct Sell {
    int64_t nrows = 0;      // valid rows
    int64_t nslices = 0;
    DBuf<int32_t> rows;     // [nslices*64] row ids (-1 past the end) or empty
    DBuf<int64_t> slice_ptr;
    DBuf<int32_t> slice_len;
    DBuf<int32_t> col;
    DBuf<double> val64;
    DBuf<float> val32;
    int64_t entries = 0;    // stored entries including padding
    int64_t nnz = 0;        // structural entries of the rows
};

// Block CSR pattern on the device (+ optional values).
struct BPattern {
    int64_t rows = 0, nnzb = 0;
    DBuf<int32_t> ptr, col;
};

struct Level {
    int64_t n = 0, nb = 1, B = 0, nnz = 0;
    // host copies of the input (kept for layout builds and save/load)
    std::vector<int64_t> h_ptr;
    std::vector<int32_t> h_col;
    std::vector<double> h_val;
    std::vector<int32_t> h_colour;   // supplied or computed block colours
    bool colour_given = false;
    // device CSR of A
    DBuf<int32_t> a_ptr, a_col;
    DBuf<double> a_val;
    Sell sell;                        // all rows, natural order
    std::vector<Sell> csell;          // per-colour rows (multiplicative)
    DBuf<int32_t> clist;              // blocks sorted by colour
    std::vector<int32_t> layout_colour;   // colours the colour layout was built for
    // saddle-point level (Stokes prescaling): kind per unknown, 0 velocity,
    // 1 pressure, 2 inert (scaled as a velocity); empty for an elliptic level
    DBuf<int32_t> kind;
    int stokes_l1 = 0;                // constraint rows normalised by the 1-norm (else max-norm)
    // overlapping blocks (Sec. 3.6.2): ovl_m slots per block, ovl_nodes[i][s] the
    // unknown of slot s of block i (-1 unused), the occurrences of every unknown
    // (CSR over block * m + slot) and 1 / multiplicity.  The smoothers of such a
    // level are [depth][ovl_nblk][ovl_m][ovl_m] in lam64 / lam32.
    int ovl_m = 0;
    int64_t ovl_nblk = 0;
    DBuf<int32_t> ovl_nodes, ovl_inv_ptr, ovl_inv_idx;
    DBuf<double> ovl_rtheta;
    DBuf<unsigned char> ovl_y;        // replicated workspace [nblk][m][R] (working precision)
    // stencil-repetition cache (Sec. 4): lattice point of every block (lat_dim
    // 0: none), the box map point -> block, and of the last exact fit the class
    // representatives [depth][B] (radius ell - 1 for cascade step ell) and the
    // blocks fitted per step
    int lat_dim = 0;
    int32_t lat_lo[3] = {0, 0, 0}, lat_ext[3] = {1, 1, 1};
    DBuf<int32_t> lat_xyz, lat_map, lat_rep;
    std::vector<int64_t> lat_fitted;
    // sweep launch schedule picked by the autotuner (0: the size rule)
    int tune_wgs = 0;                 // rows per workgroup: 64 or 256
    int64_t tune_grid = 0;            // workgroups (the kernels loop over the remaining tiles)
    std::vector<int64_t> cptr;        // colour offsets into clist
    int chi = 0;
    DBuf<int32_t> colour;             // device colours
    // interpolation to the next coarser level
    int64_t nc = 0, p_nnz = 0;
    double r_scale = 1.0;
    // agg_k > 0: P injects coarse unknown I into the fine unknowns
    // [agg_k*I, agg_k*(I+1)) with weight 1 (contiguous piecewise-constant
    // aggregation); the V-cycle then fuses residual+restriction and
    // interpolation+first post-sweep.
    int agg_k = 0;
    DBuf<int32_t> p_ptr, p_col, pt_ptr, pt_col;
    DBuf<double> p_val64, pt_val64;
    DBuf<float> p_val32, pt_val32;
    Sell psell, ptsell;               // P (fine rows) and P^T (coarse rows) as sliced ELLPACK
    // prescaling and smoother
    DBuf<double> w;
    int depth = 0;
    DBuf<double> lam64, lam64T;       // [depth][B][nb][nb] and per-block transposes
    DBuf<float> lam32, lam32T;
    std::vector<BPattern> patterns;   // E after every fit step
    int singular = 0;
    // direct segments: rows [n_active, n) solved with dense FP64 inverses (the
    // whole last level; trailing systems that end on this level in a batch)
    int64_t n_active = 0;
    int64_t act_slices = 0;           // SELL slices covering the active rows
    int64_t act_nnz = 0;              // entries of A in the active rows
    std::vector<int64_t> dseg;        // absolute row offsets, size ndseg + 1
    DBuf<int64_t> dseg_d, dinv_off;   // device copies: offsets and inverse offsets
    DBuf<double> dinv;                // concatenated row-major inverses
    int64_t dseg_max = 0;
    // BF16 block copies for 16x16 blocks (MFMA operand order), block-CSR of A
    DBuf<int32_t> bsr_ptr, bsr_col;
    std::vector<int32_t> h_bsr_ptr;   // host copy of bsr_ptr
    // per active block in colour order (cblk): {block row, first block, end
    // block, 0}, so a colour sweep reads one 16-byte record per block row
    DBuf<int32_t> bmeta;
    int64_t bsr_nnzb = 0;
    DBuf<unsigned short> a16, lam16, lam16T;
    DBuf<int32_t> cblk;               // active blocks grouped by colour
    std::vector<int64_t> cblk_ptr;    // colour offsets into cblk
    // V-cycle workspace (working precision), [n][nrhs]
    DBuf<char> xb, xt, bb, rr;
    // the workspace the V-cycle kernels use: the buffers above, or ranges of
    // the static scratch array during cs_vcycle_noalloc
    char *w_xb = nullptr, *w_xt = nullptr, *w_bb = nullptr, *w_rr = nullptr;
    unsigned char *w_ovl = nullptr;
};

// One level of the single-workgroup tail V-cycle (device copy of the
// pointers and sizes the V-cycle uses on that level; values in the working
// precision, cast by the kernel).
struct TailLevel {
    int64_t n, n_active, nslices, nc, nbl;   // rows, smoothed rows, their slices, coarse rows, Lambda entries per step
    const int64_t *sptr;
    const int32_t *slen, *scol;
    const void *sval, *lam, *lamT;
    void *bb, *xb, *xt;
    int depth, agg_k, nseg;
    double r_scale;
    const int64_t *dseg, *dinv_off;
    const double *dinv;
};

struct Trace {
    bool on = false;
    int mask = 0;                        // bit k: record class k
    int period = 1;                      // record every period-th launch of a class
    int64_t seen[CS_TRACE_NCLASS] = {0};
    std::vector<hipEvent_t> ev;          // pairs: ev[2k] start, ev[2k+1] end
    std::vector<int> cls;
    std::vector<int> cls_n;              // launches per recorded interval
    std::vector<double> cls_bytes;       // per recorded interval
    int run_cls = -1;                    // class being timed as a run of consecutive launches
    size_t used = 0;
    double ms[CS_TRACE_NCLASS] = {0};
    int64_t count[CS_TRACE_NCLASS] = {0};
    double bytes[CS_TRACE_NCLASS] = {0};
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<Level> lv;
    bool have_hierarchy = false, have_setup = false;
    cs_options opt{};
    int precision = CS_FP64;
    int ws_nrhs = 0, ws_prec = -1;
    bool ws_scratch = false;            // the level workspace points into the static scratch array
    double setup_ms = 0;
    int singular = 0;
    // independent systems on the finest level (a batch)
    std::vector<int64_t> sys_ptr;       // size nsys + 1
    DBuf<int64_t> sys_ptr_d;
    // batch residual norms: per-slice sums over slices inside one system, and
    // per-row squares of the n_het slices that straddle a system boundary
    DBuf<int32_t> sys_het;              // [nslices]: -1, or index of a straddling slice
    int64_t n_het = 0;
    DBuf<double> sys_spart;             // [nslices][R]
    DBuf<double> rn2;                   // [n_het*64][R]
    std::vector<int32_t> sys_iters;
    std::vector<double> sys_rel;
    // solve workspace
    DBuf<double> ir_partial, ir_norm;
    DBuf<double> cg_r, cg_p, cg_q;      // conjugate-gradient vectors [n][R] (FP64)
    DBuf<double> cg_zq, cg_pq;          // per (system, RHS): (z, q_prev); (p, q) and (p, r)
    DBuf<int32_t> cg_sys_wg;            // batch: first workgroup of every system in the flat kernels
    DBuf<double> cg_partial;            // batch: flat-kernel partial sums [workgroups][R]
    double *h_norm = nullptr;           // pinned host copy of ir_norm
    size_t h_norm_cap = 0;
    // GMRES: unnormalised basis [m+1][n][R], preconditioned vectors (flexible)
    // [m][n][R], two work vectors, reciprocal basis norms [m+1][nsys][R],
    // Hessenberg columns of two Gram-Schmidt passes and the new norm, the
    // least-squares solution [nsys][R][m], partial sums, batch workgroup table
    DBuf<double> gm_V, gm_Z, gm_w, gm_sc, gm_h, gm_y, gm_partial;
    DBuf<int32_t> gm_sys_wg;
    double *gm_host = nullptr;          // pinned host copy of gm_h
    size_t gm_host_cap = 0;
    bool fuse_transfers = true;         // use the fused aggregation kernels when agg_k > 0
    int64_t sweep_grid = int64_t(1) << 40;   // cap on workgroups of the tiled kernels (multiple of 8)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    Trace tr;
    // graph replay of the outer iterations of cs_solve / cs_solve_cg (on the
    // internal work stream; cs_set_graphs, cs_autotune or CS_GRAPHS=1)
    bool use_graphs = false;
    double tune_vcycle_ms[2] = {0.0, 0.0};   // last cs_autotune: V-cycle eager, replayed
    // set around a refinement V-cycle: its last fine-level sweep adds x_0 into
    // this FP64 vector (acc_done then true) instead of writing it
    double *acc_x64 = nullptr;
    bool acc_done = false;
    // single-workgroup tail V-cycle over the coarse levels of at most tail_rows
    // rows (0: off); its level table, valid for (tail_gen, tail_prec, tail_nrhs)
    int64_t tail_rows = 0;
    int tail_from = -1;                 // first level the tail covers (-1: none)
    DBuf<TailLevel> tail_tab;
    std::vector<TailLevel> tail_host;
    double tail_bytes = 0.0;            // algorithmic bytes of one tail launch (trace)
    std::vector<int64_t> tune_tail_rows;   // cs_autotune's candidates (0: off) and V-cycle ms
    std::vector<double> tune_tail_ms;
    uint64_t tail_gen = ~uint64_t(0);
    int tail_prec = -1, tail_nrhs = 0;
    uint64_t gen = 0;                   // bumped whenever device buffers the graph uses change
    hipStream_t work = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // CG: the next V-cycle's first level-0 sweep is issued before the host
    // reads the convergence norms (ev_norm marks their download); spec_pending
    // tells the next level-0 V-cycle that this sweep is already on the stream
    hipEvent_t ev_norm = nullptr;
    bool spec_pending = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    struct GraphKey {
        const void *b = nullptr, *x = nullptr;
        int nrhs = 0, prec = -1, mask = 0;
        uint64_t gen = 0;
        int method = -1;                // 0 refinement, 1 conjugate gradients
        bool operator==(const GraphKey &o) const {
            return b == o.b && x == o.x && nrhs == o.nrhs && prec == o.prec && mask == o.mask && gen == o.gen &&
                   method == o.method;
        }
    } gkey;
};

void graph_release(Ctx &c);

// tracing helpers (api.hip)
int trace_begin(Ctx &c, int cls, double bytes);   // returns slot or -1
// For one launch that records its own start and end (hipExtLaunchKernelGGL with
// *start / *stop, null when the launch is not sampled): the kernel's duration
// without event-packet overhead.  (Solves replayed from graphs are not traced.)
int trace_begin_launch(Ctx &c, int cls, double bytes, hipEvent_t *start, hipEvent_t *stop);
// One event pair around `launches` consecutive launches of class cls (their
// summed algorithmic bytes): the launches inside are not timed one by one.
int trace_begin_run(Ctx &c, int cls, double bytes, int launches);
void trace_end_run(Ctx &c, int slot);
double bf16_sweep_bytes(const Level &L, int colour, bool zero);
void build_bf16_meta(Ctx &c, Level &L, const std::vector<int32_t> &act);
void trace_end(Ctx &c, int slot);
void trace_flush(Ctx &c);
void trace_release(Ctx &c);

// setup.hip
void build_level_device(Ctx &c, Level &L);
void run_setup(Ctx &c, const cs_options &o);
void build_working_copies(Ctx &c);
void factor_direct(Ctx &c, Level &L);   // dense inverses of the direct segments
void build_colour_layout(Ctx &c, Level &L);
// learned level-0 cascade from Lambda~ [B][depth][nb][nb] (FP32, device; additive)
void run_setup_sketched(Ctx &c, const cs_options &o, int sk, const double *S);
void run_setup_learned(Ctx &c, const cs_options &o, const float *lam_t);
// Lambda~ of a level in the layout [B][depth][nb][nb] (FP32, device)
void prescaled_blocks(Ctx &c, Level &L, float *out);

// bf16.hip: 16x16 blocks in BF16 on the matrix cores
void build_bf16_level(Ctx &c, Level &L);
void build_bf16_smoother(Ctx &c, Level &L);
bool use_bf16(const Ctx &c, const Level &L);
void bf16_sweep(Ctx &c, const Level &L, int ell, int colour, bool reverse, bool zero, const float *b, float *x);

// solve.hip
void ensure_workspace(Ctx &c, int nrhs);
void vcycle_apply(Ctx &c, const double *b, double *x, int nrhs);
size_t vcycle_workspace_bytes(const Ctx &c, int nrhs);
void vcycle_apply_scratch(Ctx &c, const double *b, double *x, int nrhs, unsigned char *scratch);
void smooth_apply(Ctx &c, int level, bool reverse, const double *b, double *x, int nrhs);
void solve_ir(Ctx &c, const double *b, double *x, int nrhs, double rtol, int maxit, cs_info *info,
              double *history, cs_status *st);
void solve_cg(Ctx &c, const double *b, double *x, int nrhs, double rtol, int maxit, cs_info *info,
              double *history, cs_status *st);
void autotune(Ctx &c, int nrhs, double *ms_out);
void tune_graphs(Ctx &c, int nrhs, double *eager_ms, double *graph_ms);
int tail_start(const Ctx &c);
int tune_tail(Ctx &c, int nrhs, int64_t *rows, double *ms, int cap);
void stream_bandwidth(Ctx &c, int n_read, int n_write, int64_t bytes, int reps, double *gbps, double *us);
void solve_gmres(Ctx &c, const double *b, double *x, int nrhs, double rtol, int maxit, int restart, bool flexible,
                 cs_info *info, double *history, cs_status *st);

// host helpers
void build_sell(Sell &S, const std::vector<int64_t> &ptr, const std::vector<int32_t> &col,
                const std::vector<double> &val, const std::vector<int32_t> *rows, hipStream_t s, bool pad_with_row = true);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// blocks and block size of a level's smoothers (overlapping or not)
inline int64_t lam_count(const Level &L) { return L.ovl_m ? L.ovl_nblk : L.B; }
inline int64_t lam_size(const Level &L) { return L.ovl_m ? L.ovl_m : L.nb; }

}  // namespace cs

struct cs_ctx_s {
    cs::Ctx c;
};
