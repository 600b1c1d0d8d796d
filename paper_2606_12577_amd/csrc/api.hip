// C ABI of the cascading-smoother multigrid library; see include/cascade.h.
#include <cstdio>
#include <cstdlib>
#include <exception>
#include <fstream>
#include <map>
#include <mutex>

#include "cs_internal.h"
#include "mlp_internal.h"

using cs::Ctx;
using cs::Level;

// Workspace of cs_vcycle_noalloc (see the comment at register_scratch).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(CS_NOALLOC_SCRATCH_MIB) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_create_err;

template <class F>
cs_status guarded(cs_ctx ctx, F &&f) {
    if (!ctx) return CS_EINVAL;
    Ctx &c = ctx->c;
    try {
        CS_HIP(hipSetDevice(c.device));
        f(c);
        c.err.clear();
        return CS_OK;
    } catch (const cs::Error &e) {
        c.err = e.msg;
        return e.st;
    } catch (const std::bad_alloc &) {
        c.err = "host allocation failed";
        return CS_ENOMEM;
    } catch (const std::exception &e) {
        c.err = e.what();
        return CS_EDEVICE;
    }
}

void transpose_csr(int64_t n, int64_t nc, const std::vector<int64_t> &ptr, const std::vector<int32_t> &col,
                   const std::vector<double> &val, std::vector<int32_t> &tptr, std::vector<int32_t> &tcol,
                   std::vector<double> &tval) {
    tptr.assign(nc + 1, 0);
    for (int32_t c : col) tptr[c + 1]++;
    for (int64_t i = 0; i < nc; ++i) tptr[i + 1] += tptr[i];
    tcol.resize(col.size());
    tval.resize(col.size());
    std::vector<int32_t> fill(tptr.begin(), tptr.end() - 1);
    for (int64_t r = 0; r < n; ++r)
        for (int64_t k = ptr[r]; k < ptr[r + 1]; ++k) {
            int32_t o = fill[col[k]]++;
            tcol[o] = (int32_t)r;
            tval[o] = val[k];
        }
}

void need(bool ok, const std::string &msg, cs_status st = CS_EINVAL) {
    if (!ok) cs::fail(st, msg);
}

void set_level(Ctx &c, Level &L, const cs_level &in, int li, int nlev, int64_t n_next) {
    need(in.n > 0 && in.n < INT32_MAX, "level " + std::to_string(li) + ": n out of range");
    need(in.block_size >= 1 && in.n % in.block_size == 0, "level " + std::to_string(li) + ": block size must divide n");
    need(in.a_row_ptr && in.a_col && in.a_val, "level " + std::to_string(li) + ": A is missing");
    L.n = in.n;
    L.nb = in.block_size;
    L.B = in.n / in.block_size;
    L.h_ptr.assign(in.a_row_ptr, in.a_row_ptr + in.n + 1);
    need(L.h_ptr[0] == 0, "A row pointer must start at 0");
    for (int64_t r = 0; r < in.n; ++r) need(L.h_ptr[r + 1] >= L.h_ptr[r], "A row pointer must be non-decreasing");
    L.nnz = L.h_ptr[in.n];
    need(L.nnz < INT32_MAX, "A has too many entries for 32-bit offsets");
    L.h_col.assign(in.a_col, in.a_col + L.nnz);
    L.h_val.assign(in.a_val, in.a_val + L.nnz);
    // (the diagonal is checked by the prescaling at setup: elliptic levels need
    // a_kk > 0, saddle-point levels a positive viscous diagonal)
    for (int64_t r = 0; r < in.n; ++r)
        for (int64_t k = L.h_ptr[r]; k < L.h_ptr[r + 1]; ++k)
            need(L.h_col[k] >= 0 && L.h_col[k] < in.n, "A column index out of range");
    L.colour_given = in.colour != nullptr;
    L.layout_colour.clear();   // A changed: any colour layout is stale
    L.h_colour.clear();
    if (L.colour_given) {
        L.h_colour.assign(in.colour, in.colour + L.B);
        for (int32_t v : L.h_colour) need(v >= 0 && v < 4096, "colours must be in [0, 4096)");
    }
    // direct segments (trailing rows solved directly); the last level is all direct
    const std::string lvs = "level " + std::to_string(li) + ": ";
    L.dseg.clear();
    if (in.n_direct_seg > 0) {
        need(in.direct_seg_ptr != nullptr, lvs + "direct_seg_ptr missing");
        L.dseg.assign(in.direct_seg_ptr, in.direct_seg_ptr + in.n_direct_seg + 1);
        need(L.dseg.back() == in.n, lvs + "direct segments must end at n");
        for (int k = 0; k < in.n_direct_seg; ++k)
            need(L.dseg[k + 1] > L.dseg[k] && L.dseg[k + 1] - L.dseg[k] <= 8192,
                 lvs + "direct segments must be non-empty and at most 8192 rows");
        need(L.dseg[0] >= 0 && L.dseg[0] % in.block_size == 0, lvs + "direct segments must start on a block");
        if (li + 1 == nlev) need(L.dseg[0] == 0, lvs + "the last level must be solved directly in full");
    } else if (li + 1 == nlev) {
        need(in.n <= 8192, "bottom level larger than 8192 unknowns");
        L.dseg = {0, in.n};
    }
    L.n_active = L.dseg.empty() ? in.n : L.dseg[0];
    for (size_t k = 0; k + 1 < L.dseg.size(); ++k)
        for (int64_t r = L.dseg[k]; r < L.dseg[k + 1]; ++r)
            for (int64_t e = L.h_ptr[r]; e < L.h_ptr[r + 1]; ++e)
                need(L.h_col[e] >= L.dseg[k] && L.h_col[e] < L.dseg[k + 1],
                     lvs + "a direct segment couples to rows outside it");
    for (int64_t r = 0; r < L.n_active; ++r)
        for (int64_t e = L.h_ptr[r]; e < L.h_ptr[r + 1]; ++e)
            need(L.h_col[e] < L.n_active, lvs + "an active row couples to a direct segment");
    if (li + 1 < nlev) {
        need(L.n_active > 0, lvs + "no active rows on a level that is not the last");
        need(in.n_coarse == n_next, "level " + std::to_string(li) + ": n_coarse differs from the next level's n");
        need(in.p_row_ptr && in.p_col && in.p_val, "level " + std::to_string(li) + ": P is missing");
        std::vector<int64_t> pp(in.p_row_ptr, in.p_row_ptr + in.n + 1);
        need(pp[0] == 0, "P row pointer must start at 0");
        const int64_t pn = pp[in.n];
        std::vector<int32_t> pc(in.p_col, in.p_col + pn);
        std::vector<double> pv(in.p_val, in.p_val + pn);
        for (int32_t v : pc) need(v >= 0 && v < n_next, "P column index out of range");
        for (int64_t r = L.n_active; r < in.n; ++r) need(pp[r + 1] == pp[r], lvs + "P has entries in a direct row");
        L.nc = n_next;
        L.p_nnz = pn;
        L.r_scale = in.r_scale;
        // contiguous unit aggregation over the active rows: row r of P is the
        // single entry (r / k, 1)
        L.agg_k = 0;
        if (n_next > 0 && L.n_active % n_next == 0) {
            const int64_t k = L.n_active / n_next;
            bool ok = k <= 64 && 64 % k == 0 && pn == L.n_active;
            for (int64_t r = 0; ok && r < L.n_active; ++r)
                ok = pp[r + 1] - pp[r] == 1 && pc[pp[r]] == r / k && pv[pp[r]] == 1.0;
            if (ok) L.agg_k = (int)k;
        }
        std::vector<int32_t> tp, tc;
        std::vector<double> tv;
        transpose_csr(in.n, n_next, pp, pc, pv, tp, tc, tv);
        std::vector<int32_t> pp32(pp.begin(), pp.end());
        L.p_ptr.upload(pp32.data(), pp32.size(), c.stream);
        L.p_col.upload(pc.data(), pc.size(), c.stream);
        L.p_val64.upload(pv.data(), pv.size(), c.stream);
        std::vector<float> pvf(pv.begin(), pv.end());
        L.p_val32.upload(pvf.data(), pvf.size(), c.stream);
        L.pt_ptr.upload(tp.data(), tp.size(), c.stream);
        L.pt_col.upload(tc.data(), tc.size(), c.stream);
        L.pt_val64.upload(tv.data(), tv.size(), c.stream);
        std::vector<float> tvf(tv.begin(), tv.end());
        L.pt_val32.upload(tvf.data(), tvf.size(), c.stream);
        // sliced ELLPACK copies for the transfer kernels (columns of P are coarse
        // indices: pad with column 0)
        std::vector<int64_t> pp64(pp.begin(), pp.end()), tp64(tp.begin(), tp.end());
        cs::build_sell(L.psell, pp64, pc, pv, nullptr, c.stream, false);
        cs::build_sell(L.ptsell, tp64, tc, tv, nullptr, c.stream, false);
        CS_HIP(hipStreamSynchronize(c.stream));
    }
    cs::build_level_device(c, L);
}

// Workspace of cs_vcycle_noalloc: a fixed device array, one copy per GPU the
// library runs on (held until the process ends).  Host code never uses the
// array's name as an address: cs_create looks up each device's copy with
// hipGetSymbolAddress (once per device, that device current) and keeps it.
std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch;   // device -> its scratch address

// Returns false (and sets the creation error) when the lookup fails.
bool register_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch.count(device)) return true;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        g_create_err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
        return false;
    }
    g_scratch[device] = static_cast<unsigned char *>(p);
    return true;
}

unsigned char *device_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(device);
    return it == g_scratch.end() ? nullptr : it->second;
}

const uint64_t SAVE_MAGIC = 0x3150555445535343ull;  // "CSSETUP1"
const int32_t SAVE_VERSION = 4;   // 4: cs_options gained source and jacobi_omega

}  // namespace

namespace {

// Run a solve; a reduced-precision V-cycle that diverges (non-finite or
// exploding residual) is escalated (BF16 -> FP32 -> FP64) for this setup and
// the solve repeated.
template <class F>
cs_status solve_escalating(cs_ctx ctx, const double *b, double *x, int32_t maxit, double rtol, cs_info *info,
                           F &&run) {
    cs_status st = CS_OK;
    cs_status g = guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "solve before cs_setup", CS_ESTATE);
        need(b && x, "null vector");
        need(maxit >= 0 && rtol >= 0.0, "bad rtol or maxit");
        run(c, &st);
        while (st == CS_ENAN && c.precision != CS_FP64) {
            c.precision = c.precision == CS_BF16 ? CS_FP32 : CS_FP64;
            c.opt.precision = c.precision;
            st = CS_OK;
            run(c, &st);
        }
        if (info) info->precision = c.precision;
    });
    if (g != CS_OK) return g;
    if (st != CS_OK) ctx->c.err = cs_status_string(st);
    return st;
}

}  // namespace

extern "C" {

int32_t cs_abi_version(void) { return CS_ABI_VERSION; }

const char *cs_status_string(int32_t s) {
    switch (s) {
        case CS_OK: return "ok";
        case CS_EINVAL: return "invalid argument";
        case CS_ENOMEM: return "out of device memory";
        case CS_EDEVICE: return "HIP device error";
        case CS_ESINGULAR: return "singular normal equations";
        case CS_ECOLOR: return "improper colouring";
        case CS_ENOCONV: return "no convergence within maxit";
        case CS_ESTATE: return "call out of order";
        case CS_ENAN: return "NaN or Inf in the solve";
        case CS_EVERSION: return "saved setup has another version";
        case CS_EIO: return "file input/output failed";
        default: return "unknown status";
    }
}

cs_status cs_create(cs_ctx *out, int32_t device, void *stream) {
    if (!out) return CS_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        g_create_err = "no HIP device available";
        return CS_EDEVICE;
    }
    if (device < 0 || device >= ndev) {
        g_create_err = "device index out of range";
        return CS_EINVAL;
    }
    if (hipSetDevice(device) != hipSuccess) {
        g_create_err = "hipSetDevice failed";
        return CS_EDEVICE;
    }
    if (!register_scratch(device)) return CS_EDEVICE;
    cs_ctx h = new (std::nothrow) cs_ctx_s;
    if (!h) return CS_ENOMEM;
    h->c.device = device;
    h->c.stream = reinterpret_cast<hipStream_t>(stream);
    if (const char *g = std::getenv("CS_SWEEP_GRID")) {   // tuning override
        const long v = std::strtol(g, nullptr, 10);
        if (v >= 8) h->c.sweep_grid = (v / 8) * 8;
    }
    if (const char *f = std::getenv("CS_FUSE_TRANSFERS")) h->c.fuse_transfers = std::atoi(f) != 0;
    if (const char *f = std::getenv("CS_GRAPHS")) h->c.use_graphs = std::atoi(f) != 0;
    if (hipEventCreate(&h->c.ev0) != hipSuccess || hipEventCreate(&h->c.ev1) != hipSuccess ||
        hipEventCreateWithFlags(&h->c.ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->c.ev_out, hipEventDisableTiming) != hipSuccess) {
        g_create_err = "hipEventCreate failed";
        delete h;
        return CS_EDEVICE;
    }
    cs::pool_user(+1);
    *out = h;
    return CS_OK;
}

void cs_destroy(cs_ctx ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    cs::trace_release(ctx->c);
    cs::graph_release(ctx->c);
    if (ctx->c.work) {
        (void)hipStreamSynchronize(ctx->c.work);
        (void)hipStreamDestroy(ctx->c.work);
    }
    if (ctx->c.ev_in) (void)hipEventDestroy(ctx->c.ev_in);
    if (ctx->c.ev_out) (void)hipEventDestroy(ctx->c.ev_out);
    if (ctx->c.ev_norm) (void)hipEventDestroy(ctx->c.ev_norm);
    if (ctx->c.h_norm) (void)hipHostFree(ctx->c.h_norm);
    if (ctx->c.gm_host) (void)hipHostFree(ctx->c.gm_host);
    if (ctx->c.ev0) (void)hipEventDestroy(ctx->c.ev0);
    if (ctx->c.ev1) (void)hipEventDestroy(ctx->c.ev1);
    delete ctx;
    cs::pool_user(-1);
}

const char *cs_last_error(cs_ctx ctx) { return ctx ? ctx->c.err.c_str() : g_create_err.c_str(); }

cs_status cs_set_hierarchy(cs_ctx ctx, int32_t n_levels, const cs_level *levels) {
    return guarded(ctx, [&](Ctx &c) {
        need(n_levels >= 1 && levels != nullptr, "need at least one level");
        c.have_setup = false;
        c.have_hierarchy = false;
        c.ws_nrhs = 0;
        cs::graph_release(c);
        c.gen++;
        c.lv.clear();
        c.lv.resize(n_levels);
        for (int l = 0; l < n_levels; ++l)
            set_level(c, c.lv[l], levels[l], l, n_levels, l + 1 < n_levels ? levels[l + 1].n : 0);
        c.sys_ptr.clear();
        c.have_hierarchy = true;
    });
}

cs_status cs_setup(cs_ctx ctx, const cs_options *opt) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_hierarchy, "cs_setup before cs_set_hierarchy", CS_ESTATE);
        need(opt != nullptr, "options missing");
        need(opt->depth >= 1 && opt->depth <= 16, "depth must be in [1, 16]");
        need(opt->mode == CS_ADDITIVE || opt->mode == CS_MULTIPLICATIVE, "mode must be additive or multiplicative");
        need(opt->order == CS_FF || opt->order == CS_RF, "order must be FF or RF");
        need(opt->n_pre >= 1 && opt->n_post >= 0, "need n_pre >= 1 and n_post >= 0");
        need(opt->trunc_alpha >= 0, "trunc_alpha must be >= 0");
        need(opt->precision == CS_FP64 || opt->precision == CS_FP32 || opt->precision == CS_BF16,
             "precision must be FP64, FP32 or BF16");
        need(opt->ridge >= 0.0 && opt->ridge < 1e6, "ridge must be in [0, 1e6)");
        need(opt->source == CS_SRC_FROBENIUS || opt->source == CS_SRC_JACOBI, "source must be FROBENIUS or JACOBI");
        bool ovl = false;
        for (const Level &L : c.lv) ovl |= L.ovl_m > 0;
        if (opt->source == CS_SRC_JACOBI) {
            need(opt->jacobi_omega > 0.0 && opt->jacobi_omega <= 2.0, "jacobi_omega must be in (0, 2]");
            need(!ovl, "the block Jacobi reference smoother takes disjoint blocks");
            need(opt->trunc_alpha == 0 && opt->ridge == 0.0, "truncation and ridge apply to the fit only");
        }
        need(!ovl || (opt->mode == CS_ADDITIVE && opt->order == CS_FF && opt->trunc_alpha == 0),
             "overlapping blocks take additive cascades applied forward (FF), without truncation");
        need(!ovl || opt->ridge == 0.0, "the regularised fit does not apply to overlapping blocks");
        c.have_setup = false;
        c.opt = *opt;
        c.precision = opt->precision;
        c.ws_nrhs = 0;
        cs::run_setup(c, *opt);
        c.have_setup = true;
    });
}

cs_status cs_setup_sketched(cs_ctx ctx, const cs_options *opt, int32_t s, const double *S) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_hierarchy, "cs_setup_sketched before cs_set_hierarchy", CS_ESTATE);
        need(opt != nullptr && S != nullptr, "options or sketch missing");
        need(s >= 1 && s <= 64, "the sketch width must be in [1, 64]");
        need(opt->depth >= 1 && opt->depth <= 16, "depth must be in [1, 16]");
        need(opt->mode == CS_ADDITIVE || opt->mode == CS_MULTIPLICATIVE, "mode must be additive or multiplicative");
        need(opt->order == CS_FF || opt->order == CS_RF, "order must be FF or RF");
        need(opt->n_pre >= 1 && opt->n_post >= 0, "need n_pre >= 1 and n_post >= 0");
        need(opt->trunc_alpha == 0, "truncation applies to the exact fit only");
        need(opt->ridge == 0.0, "the regularised fit applies to the exact fit only");
        need(opt->source == CS_SRC_FROBENIUS, "the sketched construction is a Frobenius fit");
        int64_t nbmax = 1;
        for (const Level &L : c.lv) nbmax = std::max<int64_t>(nbmax, L.nb);
        // with s <= n the first level fits every sketch column exactly: T_1 = 0
        // and every later level would fit rounding noise
        bool ovl = false;
        for (const Level &L : c.lv) {
            ovl |= L.ovl_m > 0;
            if (L.ovl_m) nbmax = std::max<int64_t>(nbmax, L.ovl_m);
        }
        need(opt->depth == 1 || s > nbmax, "a deeper sketched cascade needs more sketch columns than the block size");
        need(!ovl || (opt->mode == CS_ADDITIVE && opt->order == CS_FF),
             "overlapping blocks take additive cascades applied forward (FF)");
        need(opt->precision == CS_FP64 || opt->precision == CS_FP32 || opt->precision == CS_BF16,
             "precision must be FP64, FP32 or BF16");
        c.have_setup = false;
        c.opt = *opt;
        c.precision = opt->precision;
        c.ws_nrhs = 0;
        cs::run_setup_sketched(c, *opt, s, S);
        c.have_setup = true;
    });
}

cs_status cs_setup_learned(cs_ctx ctx, const cs_options *opt, cs_mlp mlp, const float *X) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_hierarchy, "cs_setup_learned before cs_set_hierarchy", CS_ESTATE);
        need(opt != nullptr && mlp != nullptr && X != nullptr, "options, network or features missing");
        need(opt->depth >= 1 && opt->depth <= 16, "depth must be in [1, 16]");
        need(opt->mode == CS_ADDITIVE, "the learned setup fits additive cascades");
        need(opt->source == CS_SRC_FROBENIUS, "the learned setup's coarse levels are Frobenius fits");
        need(opt->ridge >= 0.0 && opt->ridge < 1e6, "ridge must be in [0, 1e6)");
        need(opt->order == CS_FF || opt->order == CS_RF, "order must be FF or RF");
        need(opt->n_pre >= 1 && opt->n_post >= 0, "need n_pre >= 1 and n_post >= 0");
        need(opt->precision == CS_FP64 || opt->precision == CS_FP32 || opt->precision == CS_BF16,
             "precision must be FP64, FP32 or BF16");
        need(c.lv.size() >= 2, "the hierarchy has no smoothed level");
        Level &L0 = c.lv[0];
        cs::Mlp &m = mlp->m;
        need(m.device == c.device, "network and context live on different devices");
        need(m.n_out == opt->depth * L0.nb * L0.nb, "network outputs must equal depth * block_size^2");
        need(L0.n_active == L0.n, "the finest level must not hold direct segments");
        c.have_setup = false;
        c.opt = *opt;
        c.precision = opt->precision;
        c.ws_nrhs = 0;
        cs::DBuf<float> lt((size_t)L0.B * m.n_out);
        CS_HIP(hipEventRecord(c.ev0, c.stream));
        cs::mlp_predict(m, c.stream, X, L0.B, lt.get());
        cs::run_setup_learned(c, *opt, lt.get());
        CS_HIP(hipEventRecord(c.ev1, c.stream));
        CS_HIP(hipEventSynchronize(c.ev1));
        float ms = 0;
        CS_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
        c.setup_ms = ms;
        c.have_setup = true;
    });
}

cs_status cs_get_prescaled_blocks(cs_ctx ctx, int32_t level, float *out) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "no setup", CS_ESTATE);
        need(level >= 0 && level + 1 < (int)c.lv.size(), "level has no smoother");
        need(out != nullptr, "null output");
        cs::prescaled_blocks(c, c.lv[level], out);
    });
}

cs_status cs_set_precision(cs_ctx ctx, int32_t precision) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "cs_set_precision before cs_setup", CS_ESTATE);
        need(precision == CS_FP64 || precision == CS_FP32 || precision == CS_BF16,
             "precision must be FP64, FP32 or BF16");
        c.precision = precision;
        c.opt.precision = precision;
    });
}

cs_status cs_get_smoother(cs_ctx ctx, int32_t level, int32_t ell, double *out) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "no setup", CS_ESTATE);
        need(level >= 0 && level + 1 < (int)c.lv.size(), "level has no smoother");
        Level &L = c.lv[level];
        need(ell >= 1 && ell <= L.depth && out, "ell out of range");
        const size_t nbl = cs::lam_count(L) * cs::lam_size(L) * cs::lam_size(L);
        CS_HIP(hipMemcpyAsync(out, L.lam64.get() + (ell - 1) * nbl, nbl * sizeof(double), hipMemcpyDeviceToHost,
                              c.stream));
        CS_HIP(hipStreamSynchronize(c.stream));
    });
}

cs_status cs_set_smoother(cs_ctx ctx, int32_t level, int32_t ell, const double *blocks) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "no setup", CS_ESTATE);
        need(level >= 0 && level + 1 < (int)c.lv.size(), "level has no smoother");
        Level &L = c.lv[level];
        need(ell >= 1 && ell <= L.depth && blocks, "ell out of range");
        const size_t nbl = cs::lam_count(L) * cs::lam_size(L) * cs::lam_size(L);
        CS_HIP(hipMemcpyAsync(L.lam64.get() + (ell - 1) * nbl, blocks, nbl * sizeof(double), hipMemcpyHostToDevice,
                              c.stream));
        cs::build_working_copies(c);
    });
}

cs_status cs_get_pattern_size(cs_ctx ctx, int32_t level, int32_t step, int64_t *nnzb) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "no setup", CS_ESTATE);
        need(level >= 0 && level + 1 < (int)c.lv.size(), "level has no smoother");
        Level &L = c.lv[level];
        need(step >= 0 && step < (int)L.patterns.size() && nnzb, "step out of range");
        *nnzb = L.patterns[step].nnzb;
    });
}

cs_status cs_get_pattern(cs_ctx ctx, int32_t level, int32_t step, int64_t *row_ptr, int32_t *col) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "no setup", CS_ESTATE);
        need(level >= 0 && level + 1 < (int)c.lv.size(), "level has no smoother");
        Level &L = c.lv[level];
        need(step >= 0 && step < (int)L.patterns.size() && row_ptr && col, "step out of range");
        const cs::BPattern &p = L.patterns[step];
        std::vector<int32_t> hp(p.rows + 1);
        p.ptr.download(hp.data(), p.rows + 1, c.stream);
        p.col.download(col, p.nnzb, c.stream);
        CS_HIP(hipStreamSynchronize(c.stream));
        for (int64_t i = 0; i <= p.rows; ++i) row_ptr[i] = hp[i];
    });
}

cs_status cs_get_colours(cs_ctx ctx, int32_t level, int32_t *out) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "no setup", CS_ESTATE);
        need(level >= 0 && level + 1 < (int)c.lv.size() && out, "level has no smoother");
        Level &L = c.lv[level];
        need(c.opt.mode == CS_MULTIPLICATIVE, "colours exist in multiplicative mode only", CS_ESTATE);
        std::copy(L.h_colour.begin(), L.h_colour.end(), out);
    });
}

cs_status cs_smooth(cs_ctx ctx, int32_t level, int32_t reverse, const double *b, double *x, int32_t nrhs) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "no setup", CS_ESTATE);
        need(level >= 0 && level + 1 < (int)c.lv.size(), "level has no smoother");
        need(b && x, "null vector");
        cs::smooth_apply(c, level, reverse != 0, b, x, nrhs);
        CS_HIP(hipStreamSynchronize(c.stream));
    });
}

cs_status cs_vcycle(cs_ctx ctx, const double *b, double *x, int32_t nrhs) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "cs_vcycle before cs_setup", CS_ESTATE);
        need(b && x, "null vector");
        cs::vcycle_apply(c, b, x, nrhs);
        CS_HIP(hipStreamSynchronize(c.stream));
    });
}

cs_status cs_vcycle_noalloc(cs_ctx ctx, const double *b, double *x, int32_t nrhs) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "cs_vcycle_noalloc before cs_setup", CS_ESTATE);
        need(b && x, "null vector");
        need(nrhs == 1 || nrhs == 2 || nrhs == 4 || nrhs == 8, "nrhs must be 1, 2, 4 or 8");
        const size_t want = cs::vcycle_workspace_bytes(c, nrhs);
        need(want <= NOALLOC_SCRATCH_BYTES,
             "cs_vcycle_noalloc needs " + std::to_string(want) + " bytes of workspace; the static scratch holds " +
                 std::to_string(NOALLOC_SCRATCH_BYTES));
        unsigned char *p = device_scratch(c.device);
        need(p != nullptr, "no scratch address for this device", CS_EDEVICE);
        cs::vcycle_apply_scratch(c, b, x, nrhs, p);
    });
}

cs_status cs_solve(cs_ctx ctx, const double *b, double *x, int32_t nrhs, double rtol, int32_t maxit, cs_info *info,
                   double *history) {
    return solve_escalating(ctx, b, x, maxit, rtol, info, [&](Ctx &c, cs_status *st) {
        cs::solve_ir(c, b, x, nrhs, rtol, maxit, info, history, st);
    });
}

cs_status cs_solve_cg(cs_ctx ctx, const double *b, double *x, int32_t nrhs, double rtol, int32_t maxit,
                      cs_info *info, double *history) {
    return solve_escalating(ctx, b, x, maxit, rtol, info, [&](Ctx &c, cs_status *st) {
        cs::solve_cg(c, b, x, nrhs, rtol, maxit, info, history, st);
    });
}

cs_status cs_set_overlapping_blocks(cs_ctx ctx, int32_t level, int64_t n_blocks, int32_t m, const int32_t *nodes) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_hierarchy, "cs_set_overlapping_blocks before cs_set_hierarchy", CS_ESTATE);
        need(level >= 0 && level + 1 < (int32_t)c.lv.size(), "level has no smoother");
        Level &L = c.lv[level];
        c.have_setup = false;
        L.depth = 0;
        if (!nodes) {
            L.ovl_m = 0;
            L.ovl_nblk = 0;
            return;
        }
        need(m >= 1 && m <= 16 && n_blocks >= 1, "need 1 <= m <= 16 slots and at least one block");
        need(L.n_active == L.n, "overlapping blocks need a level without direct segments");
        std::vector<int32_t> cnt(L.n + 1, 0);
        for (int64_t e = 0; e < n_blocks * m; ++e) {
            need(nodes[e] >= -1 && nodes[e] < L.n, "block node out of range");
            if (nodes[e] >= 0) cnt[nodes[e] + 1]++;
        }
        for (int64_t k = 0; k < L.n; ++k) need(cnt[k + 1] > 0, "every unknown must lie in some block");
        for (int64_t k = 0; k < L.n; ++k) cnt[k + 1] += cnt[k];
        std::vector<int32_t> idx(cnt[L.n]), fill(cnt.begin(), cnt.end() - 1);
        std::vector<double> rt(L.n);
        for (int64_t e = 0; e < n_blocks * m; ++e)
            if (nodes[e] >= 0) idx[fill[nodes[e]]++] = (int32_t)e;   // ascending (block, slot)
        for (int64_t k = 0; k < L.n; ++k) rt[k] = 1.0 / (cnt[k + 1] - cnt[k]);
        L.ovl_m = m;
        L.ovl_nblk = n_blocks;
        L.ovl_nodes.upload(nodes, n_blocks * m, c.stream);
        L.ovl_inv_ptr.upload(cnt.data(), cnt.size(), c.stream);
        L.ovl_inv_idx.upload(idx.data(), idx.size(), c.stream);
        L.ovl_rtheta.upload(rt.data(), rt.size(), c.stream);
        c.ws_nrhs = 0;
        CS_HIP(hipStreamSynchronize(c.stream));
    });
}

cs_status cs_set_saddle_point(cs_ctx ctx, int32_t level, const int32_t *kind, int32_t l1) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_hierarchy, "cs_set_saddle_point before cs_set_hierarchy", CS_ESTATE);
        need(level >= 0 && level < (int32_t)c.lv.size(), "level out of range");
        need(l1 == 0 || l1 == 1, "l1 must be 0 (max-norm) or 1 (1-norm)");
        Level &L = c.lv[level];
        c.have_setup = false;
        L.w.release();
        if (!kind) {
            L.kind.release();
            return;
        }
        bool any_p = false;
        for (int64_t i = 0; i < L.n; ++i) {
            need(kind[i] >= 0 && kind[i] <= 2, "kind must be 0 (velocity), 1 (pressure) or 2 (inert)");
            any_p |= kind[i] == 1;
        }
        need(any_p, "a saddle-point level needs pressure unknowns");
        L.kind.upload(kind, L.n, c.stream);
        L.stokes_l1 = l1;
        CS_HIP(hipStreamSynchronize(c.stream));
    });
}

cs_status cs_set_lattice(cs_ctx ctx, int32_t level, int32_t dim, const int32_t *coords) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_hierarchy, "cs_set_lattice before cs_set_hierarchy", CS_ESTATE);
        need(level >= 0 && level + 1 < (int32_t)c.lv.size(), "level has no smoother");
        Level &L = c.lv[level];
        if (!coords) {
            L.lat_dim = 0;
            L.lat_xyz.release();
            L.lat_map.release();
            return;
        }
        need(dim >= 1 && dim <= 3, "lattice dimension must be 1, 2 or 3");
        const int64_t B = L.B;
        constexpr int32_t LIM = 1 << 28;
        int32_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int d = 0; d < dim; ++d) {
            lo[d] = INT32_MAX;
            hi[d] = INT32_MIN;
        }
        for (int64_t b = 0; b < B; ++b)
            for (int d = 0; d < dim; ++d) {
                const int32_t v = coords[b * dim + d];
                need(v > -LIM && v < LIM, "lattice coordinates must lie in (-2^28, 2^28)");
                lo[d] = std::min(lo[d], v);
                hi[d] = std::max(hi[d], v);
            }
        int32_t ext[3] = {1, 1, 1};
        int64_t vol = 1;
        for (int d = 0; d < dim; ++d) {
            ext[d] = hi[d] - lo[d] + 1;
            vol *= ext[d];
            need(vol <= (int64_t)LIM, "bounding box of the lattice points above 2^28 points");
        }
        std::vector<int32_t> map((size_t)vol, -1), xyz((size_t)B * 3, 0);
        for (int64_t b = 0; b < B; ++b) {
            int64_t idx = 0;
            for (int d = dim - 1; d >= 0; --d) {
                const int32_t v = coords[b * dim + d];
                xyz[(size_t)b * 3 + d] = v;
                idx = idx * ext[d] + (v - lo[d]);
            }
            need(map[(size_t)idx] < 0, "lattice points must be distinct");
            map[(size_t)idx] = (int32_t)b;
        }
        L.lat_xyz.upload(xyz.data(), xyz.size(), c.stream);
        L.lat_map.upload(map.data(), map.size(), c.stream);
        for (int d = 0; d < 3; ++d) {
            L.lat_lo[d] = lo[d];
            L.lat_ext[d] = ext[d];
        }
        L.lat_dim = dim;
        CS_HIP(hipStreamSynchronize(c.stream));
    });
}

cs_status cs_get_lattice_stats(cs_ctx ctx, int32_t level, int64_t *fitted, int32_t *rep) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "no setup", CS_ESTATE);
        need(level >= 0 && level + 1 < (int32_t)c.lv.size() && fitted, "level has no smoother");
        Level &L = c.lv[level];
        need(L.lat_fitted.size() == (size_t)L.depth, "the last setup of this level was not an exact block fit",
             CS_ESTATE);
        std::copy(L.lat_fitted.begin(), L.lat_fitted.end(), fitted);
        if (!rep) return;
        const size_t B = (size_t)L.B;
        if (L.lat_rep.get()) {
            L.lat_rep.download(rep, (size_t)L.depth * B, c.stream);
            CS_HIP(hipStreamSynchronize(c.stream));
        } else {
            for (int e = 0; e < L.depth; ++e)
                for (size_t b = 0; b < B; ++b) rep[e * B + b] = (int32_t)b;
        }
    });
}

cs_status cs_autotune(cs_ctx ctx, int32_t nrhs, int32_t *wgs, int64_t *grid, double *ms) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "autotune before cs_setup", CS_ESTATE);
        need(nrhs == 1 || nrhs == 2 || nrhs == 4 || nrhs == 8, "nrhs must be 1, 2, 4 or 8");
        cs::autotune(c, nrhs, ms);
        for (size_t l = 0; l < c.lv.size(); ++l) {
            if (wgs) wgs[l] = c.lv[l].tune_wgs;
            if (grid) grid[l] = c.lv[l].tune_grid;
        }
        c.tune_tail_rows.assign(c.lv.size() + 1, 0);
        c.tune_tail_ms.assign(c.lv.size() + 1, 0.0);
        const int nt = cs::tune_tail(c, nrhs, c.tune_tail_rows.data(), c.tune_tail_ms.data(), (int)c.lv.size() + 1);
        c.tune_tail_rows.resize(nt);
        c.tune_tail_ms.resize(nt);
        double e = 0.0, g = 0.0;
        cs::tune_graphs(c, nrhs, &e, &g);
        c.tune_vcycle_ms[0] = e;
        c.tune_vcycle_ms[1] = g;
    });
}

cs_status cs_set_graphs(cs_ctx ctx, int32_t on) {
    return guarded(ctx, [&](Ctx &c) {
        need(on == 0 || on == 1, "graph replay is 0 (off) or 1 (on)");
        c.use_graphs = on != 0;
    });
}

cs_status cs_get_graphs(cs_ctx ctx, int32_t *on, double *eager_ms, double *graph_ms) {
    return guarded(ctx, [&](Ctx &c) {
        need(on != nullptr, "null output");
        *on = c.use_graphs ? 1 : 0;
        if (eager_ms) *eager_ms = c.tune_vcycle_ms[0];
        if (graph_ms) *graph_ms = c.tune_vcycle_ms[1];
    });
}

cs_status cs_set_tail(cs_ctx ctx, int64_t max_rows) {
    return guarded(ctx, [&](Ctx &c) {
        need(max_rows >= 0 && max_rows <= 65536, "tail max_rows must be in [0, 65536]");
        c.tail_rows = max_rows;
        c.tail_from = -1;
        c.tail_gen = ~uint64_t(0);   // rebuilt by the next V-cycle
        c.gen++;                     // captured graphs hold the old launch sequence
    });
}

cs_status cs_get_tail(cs_ctx ctx, int64_t *max_rows, int32_t *first_level, int32_t cap, int64_t *cand_rows,
                      double *cand_ms, int32_t *n_cand) {
    return guarded(ctx, [&](Ctx &c) {
        need(max_rows != nullptr && first_level != nullptr, "null output");
        need(cap >= 0 && (cap == 0 || (cand_rows != nullptr && cand_ms != nullptr)), "candidate arrays");
        *max_rows = c.tail_rows;
        *first_level = c.have_setup ? cs::tail_start(c) : -1;
        const int nt = (int)c.tune_tail_rows.size();
        for (int k = 0; k < std::min(nt, (int)cap); ++k) {
            cand_rows[k] = c.tune_tail_rows[k];
            cand_ms[k] = c.tune_tail_ms[k];
        }
        if (n_cand) *n_cand = nt;
    });
}

cs_status cs_stream_bandwidth(cs_ctx ctx, int32_t n_read, int32_t n_write, int64_t bytes, int32_t reps,
                              double *gbps, double *us) {
    return guarded(ctx, [&](Ctx &c) { cs::stream_bandwidth(c, n_read, n_write, bytes, reps, gbps, us); });
}

cs_status cs_solve_gmres(cs_ctx ctx, const double *b, double *x, int32_t nrhs, double rtol, int32_t maxit,
                         int32_t restart, int32_t flexible, cs_info *info, double *history) {
    return solve_escalating(ctx, b, x, maxit, rtol, info, [&](Ctx &c, cs_status *st) {
        cs::solve_gmres(c, b, x, nrhs, rtol, maxit, restart, flexible != 0, info, history, st);
    });
}

cs_status cs_save_setup(cs_ctx ctx, const char *path) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_setup, "no setup", CS_ESTATE);
        need(path != nullptr, "null path");
        std::ofstream f(path, std::ios::binary);
        need((bool)f, std::string("cannot open ") + path, CS_EIO);
        auto put = [&](const void *p, size_t n) { f.write(reinterpret_cast<const char *>(p), (std::streamsize)n); };
        put(&SAVE_MAGIC, 8);
        put(&SAVE_VERSION, 4);
        put(&c.opt, sizeof(c.opt));
        int32_t nl = (int32_t)c.lv.size();
        put(&nl, 4);
        for (size_t l = 0; l < c.lv.size(); ++l) {
            Level &L = c.lv[l];
            int64_t hdr[3] = {L.n, L.nb, (int64_t)L.h_colour.size()};
            put(hdr, sizeof(hdr));
            put(L.h_colour.data(), L.h_colour.size() * 4);
            std::vector<double> buf;
            if (l + 1 < c.lv.size()) {
                buf.resize((size_t)L.depth * L.B * L.nb * L.nb);
                L.lam64.download(buf.data(), buf.size(), c.stream);
            }
            std::vector<double> dbuf(L.dinv.n);
            L.dinv.download(dbuf.data(), dbuf.size(), c.stream);
            CS_HIP(hipStreamSynchronize(c.stream));
            int64_t cnt = (int64_t)buf.size();
            put(&cnt, 8);
            put(buf.data(), buf.size() * 8);
            cnt = (int64_t)dbuf.size();
            put(&cnt, 8);
            put(dbuf.data(), dbuf.size() * 8);
        }
        need((bool)f, std::string("write failed: ") + path, CS_EIO);
    });
}

cs_status cs_load_setup(cs_ctx ctx, const char *path) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_hierarchy, "cs_load_setup before cs_set_hierarchy", CS_ESTATE);
        need(path != nullptr, "null path");
        std::ifstream f(path, std::ios::binary);
        need((bool)f, std::string("cannot open ") + path, CS_EIO);
        auto get = [&](void *p, size_t n) {
            f.read(reinterpret_cast<char *>(p), (std::streamsize)n);
            need((bool)f, "truncated setup file", CS_EIO);
        };
        uint64_t magic = 0;
        int32_t ver = 0;
        get(&magic, 8);
        need(magic == SAVE_MAGIC, "not a setup file", CS_EIO);
        get(&ver, 4);
        need(ver == SAVE_VERSION, "setup file version mismatch", CS_EVERSION);
        cs_options o;
        get(&o, sizeof(o));
        int32_t nl = 0;
        get(&nl, 4);
        need(nl == (int32_t)c.lv.size(), "setup file is for another hierarchy");
        c.have_setup = false;
        for (int l = 0; l < nl; ++l) {
            Level &L = c.lv[l];
            int64_t hdr[3];
            get(hdr, sizeof(hdr));
            need(hdr[0] == L.n && hdr[1] == L.nb, "setup file is for another hierarchy");
            need(hdr[2] >= 0 && hdr[2] <= L.B, "bad colour count in setup file", CS_EIO);
            L.h_colour.resize(hdr[2]);
            get(L.h_colour.data(), hdr[2] * 4);
            int64_t cnt = 0;
            get(&cnt, 8);
            std::vector<double> buf(cnt);
            get(buf.data(), cnt * 8);
            if (l + 1 < nl) {
                need(cnt > 0 && cnt % (L.B * L.nb * L.nb) == 0, "bad smoother size in setup file", CS_EIO);
                L.depth = (int)(cnt / (L.B * L.nb * L.nb));
                L.lam64.upload(buf.data(), cnt, c.stream);
                CS_HIP(hipStreamSynchronize(c.stream));
                if (o.mode == CS_MULTIPLICATIVE) {
                    need((int64_t)L.h_colour.size() == L.B, "missing colours in setup file", CS_EIO);
                    cs::build_colour_layout(c, L);
                    L.layout_colour = L.h_colour;
                }
            }
            get(&cnt, 8);
            need(cnt == (int64_t)L.dinv.n, "bad direct-segment inverses in setup file", CS_EIO);
            buf.resize(cnt);
            get(buf.data(), cnt * 8);
            L.dinv.upload(buf.data(), cnt, c.stream);
            CS_HIP(hipStreamSynchronize(c.stream));
            L.patterns.clear();
        }
        CS_HIP(hipStreamSynchronize(c.stream));
        c.opt = o;
        c.precision = o.precision;
        c.ws_nrhs = 0;
        cs::build_working_copies(c);
        c.have_setup = true;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// tracing
// ---------------------------------------------------------------------------
namespace cs {

// A free event pair for one recorded interval of class cls covering
// `launches` launches and `bytes` algorithmic bytes.
static int trace_slot(Trace &t, int cls, double bytes, int launches) {
    if (2 * t.used + 2 > t.ev.size()) {
        hipEvent_t a, b;
        CS_HIP(hipEventCreate(&a));
        CS_HIP(hipEventCreate(&b));
        t.ev.push_back(a);
        t.ev.push_back(b);
        t.cls.push_back(0);
        t.cls_n.push_back(0);
        t.cls_bytes.push_back(0.0);
    }
    const int slot = (int)t.used++;
    t.cls[slot] = cls;
    t.cls_n[slot] = launches;
    t.cls_bytes[slot] = bytes;
    return slot;
}

static bool trace_sampled(Trace &t, int cls) {
    if (!t.on || !((t.mask >> cls) & 1) || cls == t.run_cls) return false;
    return t.seen[cls]++ % t.period == 0;
}

int trace_begin(Ctx &c, int cls, double bytes) {
    Trace &t = c.tr;
    if (!trace_sampled(t, cls)) return -1;
    const int slot = trace_slot(t, cls, bytes, 1);
    CS_HIP(hipEventRecord(t.ev[2 * slot], c.stream));
    return slot;
}

int trace_begin_launch(Ctx &c, int cls, double bytes, hipEvent_t *start, hipEvent_t *stop) {
    *start = *stop = nullptr;
    Trace &t = c.tr;
    if (!trace_sampled(t, cls)) return -1;
    const int slot = trace_slot(t, cls, bytes, 1);
    *start = t.ev[2 * slot];
    *stop = t.ev[2 * slot + 1];
    return slot;
}

int trace_begin_run(Ctx &c, int cls, double bytes, int launches) {
    Trace &t = c.tr;
    if (launches <= 0 || !trace_sampled(t, cls)) return -1;
    t.run_cls = cls;   // the launches inside are not sampled one by one
    const int slot = trace_slot(t, cls, bytes, launches);
    CS_HIP(hipEventRecord(t.ev[2 * slot], c.stream));
    return slot;
}

void trace_end_run(Ctx &c, int slot) {
    if (slot == -1) return;
    CS_HIP(hipEventRecord(c.tr.ev[2 * slot + 1], c.stream));
    c.tr.run_cls = -1;
}

void trace_end(Ctx &c, int slot) {
    if (slot == -1) return;
    CS_HIP(hipEventRecord(c.tr.ev[2 * slot + 1], c.stream));
}

void graph_release(Ctx &c) {
    if (c.gexec) (void)hipGraphExecDestroy(c.gexec);
    if (c.graph) (void)hipGraphDestroy(c.graph);
    c.gexec = nullptr;
    c.graph = nullptr;
    c.gkey = Ctx::GraphKey{};
}

void trace_flush(Ctx &c) {
    Trace &t = c.tr;
    if (t.used == 0) return;
    CS_HIP(hipStreamSynchronize(c.stream));
    for (size_t k = 0; k < t.used; ++k) {
        float ms = 0;
        CS_HIP(hipEventElapsedTime(&ms, t.ev[2 * k], t.ev[2 * k + 1]));
        t.ms[t.cls[k]] += ms;
        t.count[t.cls[k]] += t.cls_n[k];
        t.bytes[t.cls[k]] += t.cls_bytes[k];
    }
    t.used = 0;
}

void trace_release(Ctx &c) {
    for (hipEvent_t e : c.tr.ev) (void)hipEventDestroy(e);
    c.tr.ev.clear();
    c.tr.cls.clear();
    c.tr.cls_n.clear();
    c.tr.cls_bytes.clear();
    c.tr.run_cls = -1;
    c.tr.used = 0;
}

}  // namespace cs

extern "C" {

cs_status cs_trace(cs_ctx ctx, int32_t mask, int32_t period) {
    return guarded(ctx, [&](Ctx &c) {
        need(period >= 1, "trace period must be >= 1");
        cs::trace_flush(c);
        c.tr.mask = mask;
        c.tr.period = period;
        c.tr.run_cls = -1;
        const int32_t enable = mask;
        if (enable) {
            for (int k = 0; k < CS_TRACE_NCLASS; ++k) {
                c.tr.ms[k] = 0;
                c.tr.count[k] = 0;
                c.tr.bytes[k] = 0;
                c.tr.seen[k] = 0;
            }
        }
        c.tr.on = enable != 0;
    });
}

cs_status cs_trace_read(cs_ctx ctx, int32_t cls, double *total_ms, int64_t *launches, double *bytes) {
    return guarded(ctx, [&](Ctx &c) {
        need(cls >= 0 && cls < CS_TRACE_NCLASS, "trace class out of range");
        cs::trace_flush(c);
        if (total_ms) *total_ms = c.tr.ms[cls];
        if (launches) *launches = c.tr.count[cls];
        if (bytes) *bytes = c.tr.bytes[cls];
    });
}

}  // extern "C"

extern "C" {

cs_status cs_set_systems(cs_ctx ctx, int32_t nsys, const int64_t *row_ptr) {
    return guarded(ctx, [&](Ctx &c) {
        need(c.have_hierarchy, "cs_set_systems before cs_set_hierarchy", CS_ESTATE);
        need(nsys >= 1, "need at least one system");
        std::vector<int64_t> p;
        if (nsys == 1 && row_ptr == nullptr) {
            p = {0, c.lv[0].n};
        } else {
            need(row_ptr != nullptr, "row_ptr missing");
            p.assign(row_ptr, row_ptr + nsys + 1);
        }
        need(p.front() == 0 && p.back() == c.lv[0].n, "systems must cover the finest level");
        for (int s = 0; s < nsys; ++s) need(p[s + 1] > p[s], "systems must be non-empty");
        c.sys_ptr = nsys > 1 ? p : std::vector<int64_t>{};
        c.n_het = 0;
        if (nsys > 1) {
            c.sys_ptr_d.upload(c.sys_ptr.data(), c.sys_ptr.size(), c.stream);
            // 64-row slices of the finest level that hold rows of several systems
            const int64_t n = c.lv[0].n, ns = cs::ceil_div(n, 64);
            std::vector<int32_t> het(ns, -1);
            int q = 0;
            for (int64_t k = 0; k < ns; ++k) {
                const int64_t first = 64 * k, last = std::min(first + 64, n) - 1;
                while (p[q + 1] <= first) ++q;
                if (last >= p[q + 1]) het[k] = (int32_t)c.n_het++;
            }
            c.sys_het.upload(het.data(), het.size(), c.stream);
        }
        CS_HIP(hipStreamSynchronize(c.stream));
        c.ws_nrhs = 0;   // workspace depends on the system count
    });
}

cs_status cs_get_system_stats(cs_ctx ctx, int32_t *iterations, double *rel_res) {
    return guarded(ctx, [&](Ctx &c) {
        need(!c.sys_iters.empty(), "no solve with systems has run", CS_ESTATE);
        need(iterations && rel_res, "null output");
        std::copy(c.sys_iters.begin(), c.sys_iters.end(), iterations);
        std::copy(c.sys_rel.begin(), c.sys_rel.end(), rel_res);
    });
}

}  // extern "C"
