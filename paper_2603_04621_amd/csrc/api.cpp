// C ABI of libdualip: validation, create-time layout, dual evaluation and the
// single-problem solve loop.  See include/dualip.h for the contract.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "problem.hpp"

using namespace dl;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace dlh {

static thread_local std::string g_err;

void set_error(const char* fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

dl_status hip_fail(hipError_t e, const char* what)
{
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? DL_ERR_OUT_OF_MEMORY : DL_ERR_DEVICE;
}

}  // namespace dlh

using dlh::set_error;
using dlh::hip_fail;

#define HIP_TRY(call, what)                                   \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(e_, what);      \
    } while (0)

extern "C" const char* dl_last_error(void) { return dlh::g_err.c_str(); }

extern "C" const char* dl_status_str(dl_status s)
{
    switch (s) {
    case DL_OK: return "ok";
    case DL_ERR_INVALID_ARG: return "invalid argument";
    case DL_ERR_UNSUPPORTED: return "unsupported";
    case DL_ERR_OUT_OF_MEMORY: return "out of memory";
    case DL_ERR_DEVICE: return "device error";
    case DL_ERR_NUMERIC: return "numeric error";
    case DL_ERR_NOT_CONVERGED: return "not converged";
    case DL_ERR_BUSY: return "busy";
    case DL_ERR_NOT_FOUND: return "not found";
    }
    return "unknown status";
}

extern "C" void dl_problem_opts_init(dl_problem_opts* o)
{
    if (!o) return;
    o->storage = DL_F32;
    o->row_normalize = 1;
    o->primal_scale = 0;
    o->v = nullptr;
    o->autotune = 0;
    o->deterministic = 0;
    o->lane_cap = o->seg_rmax = o->wg_min = o->chunks_per_cu = 0;
}

extern "C" void dl_solve_opts_init(dl_solve_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->gamma0 = 0.01;
    o->gamma_final = 0.01;
    o->n_stages = 1;
    o->momentum = 1;
    o->stage_iters = 0;
    o->stage_tol = 0.0;
    o->tol_rel_gap = 1e-4;
    o->max_iters = 10000;
    o->check_every = 10;
    o->max_step = 0.01;
    o->init_step = 1e-4;
    o->adaptive = 1;
    o->warm_start = 0;
    o->graph_iters = 0;
    o->time_kernels = 0;
    o->trace_host = nullptr;
    o->preset = DL_PRESET_CUSTOM;
    o->reserved = 0;
}

extern "C" dl_status dl_solve_opts_apply_preset(dl_solve_opts* o, double anorm2)
{
    if (!o) { set_error("opts is NULL"); return DL_ERR_INVALID_ARG; }
    if (!(anorm2 > 0.0) || !std::isfinite(anorm2)) { set_error("anorm2 must be positive and finite"); return DL_ERR_INVALID_ARG; }
    if (!(o->gamma0 > 0.0) || !std::isfinite(o->gamma0)) { set_error("gamma0 must be positive"); return DL_ERR_INVALID_ARG; }
    // step cap and first step as fractions of 1/L at gamma0, L = |A'|^2 / gamma0
    switch (o->preset) {
    case DL_PRESET_CUSTOM: return DL_OK;
    case DL_PRESET_PAPER:
        o->max_step = 0.1 * o->gamma0 / anorm2;
        o->init_step = 1e-3 * o->gamma0 / anorm2;
        return DL_OK;
    case DL_PRESET_NATURAL:
        o->max_step = o->gamma0 / anorm2;
        o->init_step = 1e-2 * o->gamma0 / anorm2;
        return DL_OK;
    }
    set_error("unknown preset %d", (int)o->preset);
    return DL_ERR_INVALID_ARG;
}

// ---------------------------------------------------------------------------
// validation (host only)
// ---------------------------------------------------------------------------
static bool finite_all(const double* v, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

static dl_status validate_impl(const dl_problem_desc* d, const dl_problem_opts* o, int* solve_ok,
                               int* col_entries = nullptr)
{
    int maxk = d && d->n > 0 ? 1 : 0;   // largest number of entries in a column
    if (!d) { set_error("desc is NULL"); return DL_ERR_INVALID_ARG; }
    if (d->m < 1 || d->m >= (int64_t)1 << 28) { set_error("m must be in [1, 2^28)"); return DL_ERR_INVALID_ARG; }
    if (d->n < 0 || d->nnz < 0) { set_error("n and nnz must be >= 0"); return DL_ERR_INVALID_ARG; }
    if (d->layout != DL_CSC && d->layout != DL_CSR) { set_error("unknown layout %d", (int)d->layout); return DL_ERR_INVALID_ARG; }
    if (d->nnz > 0 && (!d->idx || !d->val)) { set_error("idx/val are NULL"); return DL_ERR_INVALID_ARG; }
    if (d->n > 0 && !d->c) { set_error("c is NULL"); return DL_ERR_INVALID_ARG; }
    if (!d->b) { set_error("b is NULL"); return DL_ERR_INVALID_ARG; }
    if (d->num_blocks < 0 || !d->block_off) { set_error("blocks missing"); return DL_ERR_INVALID_ARG; }
    if (d->num_blocks > 0 && !d->block_proj) { set_error("block_proj is NULL"); return DL_ERR_INVALID_ARG; }
    if (d->block_off[0] != 0 || d->block_off[d->num_blocks] != d->n) {
        set_error("block_off must start at 0 and end at n"); return DL_ERR_INVALID_ARG;
    }
    for (int64_t i = 0; i < d->num_blocks; ++i) {
        if (d->block_off[i + 1] < d->block_off[i]) { set_error("block_off decreases at %lld", (long long)i); return DL_ERR_INVALID_ARG; }
        if (d->block_proj[i] > DL_PROJ_CAPPED) { set_error("block_proj[%lld] = %d is not a dl_proj", (long long)i, (int)d->block_proj[i]); return DL_ERR_INVALID_ARG; }
        if (d->block_off[i + 1] - d->block_off[i] >= (int64_t)1 << 31) { set_error("block too large"); return DL_ERR_UNSUPPORTED; }
    }
    if (!finite_all(d->val, d->nnz)) { set_error("val has a non-finite entry"); return DL_ERR_INVALID_ARG; }
    if (!finite_all(d->c, d->n)) { set_error("c has a non-finite entry"); return DL_ERR_INVALID_ARG; }
    if (!finite_all(d->b, d->m)) { set_error("b has a non-finite entry"); return DL_ERR_INVALID_ARG; }
    if (d->upper)
        for (int64_t e = 0; e < d->n; ++e)
            if (std::isnan(d->upper[e]) || d->upper[e] < 0.0) { set_error("upper[%lld] must be >= 0", (long long)e); return DL_ERR_INVALID_ARG; }
    if (d->layout == DL_CSC) {
        if (!d->ptr) {
            if (d->nnz != d->n) { set_error("CSC with ptr = NULL needs nnz == n"); return DL_ERR_INVALID_ARG; }
        } else {
            if (d->ptr[0] != 0 || d->ptr[d->n] != d->nnz) { set_error("CSC ptr must run from 0 to nnz"); return DL_ERR_INVALID_ARG; }
            for (int64_t e = 0; e < d->n; ++e) {
                const int64_t k = d->ptr[e + 1] - d->ptr[e];
                if (k < 0) { set_error("CSC ptr decreases at column %lld", (long long)e); return DL_ERR_INVALID_ARG; }
                if (k > kMfPlanes) { set_error("column %lld has %lld entries: at most %d are supported", (long long)e, (long long)k, kMfPlanes); return DL_ERR_UNSUPPORTED; }
                maxk = std::max<int>(maxk, (int)k);
            }
        }
        for (int64_t k = 0; k < d->nnz; ++k)
            if (d->idx[k] < 0 || d->idx[k] >= d->m) { set_error("row index %d out of range at %lld", d->idx[k], (long long)k); return DL_ERR_INVALID_ARG; }
    } else {
        if (!d->ptr) { set_error("CSR needs ptr"); return DL_ERR_INVALID_ARG; }
        if (d->ptr[0] != 0 || d->ptr[d->m] != d->nnz) { set_error("CSR ptr must run from 0 to nnz"); return DL_ERR_INVALID_ARG; }
        for (int64_t j = 0; j < d->m; ++j)
            if (d->ptr[j + 1] < d->ptr[j]) { set_error("CSR ptr decreases at row %lld", (long long)j); return DL_ERR_INVALID_ARG; }
        std::vector<uint8_t> seen((size_t)d->n, 0);
        for (int64_t k = 0; k < d->nnz; ++k) {
            const int32_t e = d->idx[k];
            if (e < 0 || e >= d->n) { set_error("column index %d out of range at %lld", e, (long long)k); return DL_ERR_INVALID_ARG; }
            if (seen[e] >= kMfPlanes) { set_error("column %d has more than %d entries", e, kMfPlanes); return DL_ERR_UNSUPPORTED; }
            maxk = std::max<int>(maxk, ++seen[e]);
        }
    }
    if (o) {
        if (o->storage < DL_F64 || o->storage > DL_BF16_AC) { set_error("unknown storage %d", (int)o->storage); return DL_ERR_INVALID_ARG; }
        if (o->row_normalize != 0 && o->row_normalize != 1) { set_error("row_normalize must be 0 or 1"); return DL_ERR_INVALID_ARG; }
        if (o->primal_scale < 0 || o->primal_scale > 2) { set_error("primal_scale must be 0, 1 or 2"); return DL_ERR_INVALID_ARG; }
        if (o->deterministic != 0 && o->deterministic != 1) { set_error("deterministic must be 0 or 1"); return DL_ERR_INVALID_ARG; }
        if (o->deterministic && maxk > 1) { set_error("deterministic mode supports one entry per column only"); return DL_ERR_UNSUPPORTED; }
        if (o->lane_cap < 0 || o->seg_rmax < 0 || o->wg_min < 0 || o->chunks_per_cu < 0 || o->chunks_per_cu > 8) {
            set_error("layout fields must be >= 0 (chunks_per_cu <= 8)"); return DL_ERR_INVALID_ARG;
        }
        if (o->primal_scale == 2) {
            if (!o->v) { set_error("primal_scale = 2 needs v"); return DL_ERR_INVALID_ARG; }
            for (int64_t e = 0; e < d->n; ++e)
                if (!(o->v[e] > 0.0) || !std::isfinite(o->v[e])) { set_error("v[%lld] must be positive and finite", (long long)e); return DL_ERR_INVALID_ARG; }
        }
    }
    int ok = 1;
    for (int64_t k = 0; k < d->nnz && ok; ++k) ok = d->val[k] >= 0.0;
    for (int64_t j = 0; j < d->m && ok; ++j) ok = d->b[j] >= 0.0;
    if (solve_ok) *solve_ok = ok;
    if (col_entries) *col_entries = maxk;
    return DL_OK;
}

extern "C" dl_status dl_problem_validate(const dl_problem_desc* d, const dl_problem_opts* o)
{
    return validate_impl(d, o, nullptr);
}

dl_status dlh::validate_desc(const dl_problem_desc* d, const dl_problem_opts* o, int* col_entries)
{
    return validate_impl(d, o, nullptr, col_entries);
}

// ---------------------------------------------------------------------------
// create: host layout
// ---------------------------------------------------------------------------
static uint16_t to_bf16(double x)
{
    const float f = (float)x;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

template <typename F>
static void parallel_for(int64_t n, int64_t grain, F f)
{
    int nt = (int)std::min<int64_t>(16, std::max<int64_t>(1, n / std::max<int64_t>(grain, 1)));
    nt = std::max(1, std::min<int>(nt, (int)std::thread::hardware_concurrency()));
    if (nt <= 1) {
        f(0, n);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
        const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
        th.emplace_back([=]() { f(lo, hi); });
    }
    for (auto& x : th) x.join();
}

struct HostLayout {
    std::vector<Item> items;
    std::vector<Chunk> chunks;
    std::vector<int64_t> src;      // stream position -> original column
    int64_t n_lane = 0, n_seg = 0, n_wg = 0;   // one-lane groups, multi-lane groups, WG blocks
};

// Lanes per block (log2) of a block of d edges: 0 up to cap, else -1 (a WG
// block) from wgmin edges on (wgmin > 0); else, among S = 2^lg (lg = 1..6,
// or 2, 4, 6 when even) with R = ceil(d / S) <= rmax rows per lane, the S
// whose register rows pad the block least: the kernel holds R rows in a
// class of 4 rows (R <= 4, when p4: the multi-entry kernel), 8 rows (R <= 8)
// or pmax rows, so a group costs S times the class in row slots (the smaller
// S on ties: fewer reduction steps); -1 for longer blocks.
static int block_lg(int64_t d, int cap, int rmax, int pmax, bool even, int wgmin, bool p4)
{
    if (d <= cap) return 0;
    if (wgmin > 0 && d >= wgmin) return -1;
    int best = -1;
    int64_t best_slots = 0;
    for (int lg = even ? 2 : 1; lg <= 6; lg += even ? 2 : 1) {
        const int64_t R = (d + (1 << lg) - 1) >> lg;
        if (R > rmax) continue;
        const int64_t slots = ((int64_t)1 << lg) * (p4 && R <= 4 ? 4 : R <= 8 ? 8 : pmax);
        if (best < 0 || slots < best_slots) {
            best = lg;
            best_slots = slots;
        }
    }
    return best;
}

// Groups blocks by (lanes per block, projection, degree), deals the work
// items of each kind round-robin to the chunks (in that order, so every
// chunk gets the same mix of sizes and the same share of nonzeros: a chunk's
// time follows its number of items as much as its nonzeros; WG blocks, few
// and of very different sizes, go in decreasing size with the direction of
// the deal reversed every round) and lays the stream out chunk by chunk, so
// each workgroup reads one contiguous region per kind.
static void build_items(const dl_problem_desc* d, int nchunks, int cap, int rmax, int pmax, bool even, int wgmin,
                        bool p4, HostLayout& L)
{
    const int64_t I = d->num_blocks;
    const int64_t dmax_lane = std::max<int64_t>(cap, 64 * (int64_t)rmax);
    // buckets: [lg][proj][degree] for LANE items, then WG blocks by proj
    constexpr int NPJ = 3;   // projection types (dl_proj)
    std::vector<std::vector<int64_t>> lane((size_t)7 * NPJ * (dmax_lane + 1));
    auto bucket = [&](int lg, int pr, int64_t deg) -> std::vector<int64_t>& {
        return lane[((size_t)lg * NPJ + pr) * (dmax_lane + 1) + deg];
    };
    std::vector<std::pair<int64_t, int64_t>> wgb;   // (proj, block)
    for (int64_t i = 0; i < I; ++i) {
        const int64_t deg = d->block_off[i + 1] - d->block_off[i];
        const int pr = d->block_proj[i];
        if (deg == 0) continue;
        // capped-simplex blocks: smaller one-lane and per-lane classes
        const int lg = pr == DL_PROJ_CAPPED
                           ? block_lg(deg, std::min(cap, kCutLaneCap), std::min(rmax, kCutRmax),
                                      std::min(pmax, kCutRmax), even, wgmin, p4)
                           : block_lg(deg, cap, rmax, pmax, even, wgmin, p4);
        if (lg >= 0) bucket(lg, pr, deg).push_back(i);
        else wgb.push_back({(int64_t)pr, i});
    }
    // WG blocks by projection, then by decreasing degree (dealt below in a
    // serpentine so every chunk gets the same share of their nonzeros)
    auto bdeg = [&](int64_t i) { return d->block_off[i + 1] - d->block_off[i]; };
    std::stable_sort(wgb.begin(), wgb.end(), [&](auto& a, auto& b) {
        if (a.first != b.first) return a.first < b.first;
        return bdeg(a.second) > bdeg(b.second);
    });

    // items of each kind in order; gb holds their blocks
    struct Proto {
        Item it;
        int64_t g0;   // first block in gb
    };
    std::vector<Proto> kinds[2];
    std::vector<int64_t> gb;
    for (int lg = 0; lg <= 6; ++lg)
        for (int pr = 0; pr < NPJ; ++pr)
            for (int64_t deg = 1; deg <= dmax_lane; ++deg) {
                const auto& v = bucket(lg, pr, deg);
                const size_t per = (size_t)64 >> lg;
                for (size_t s0 = 0; s0 < v.size(); s0 += per) {
                    const int nb = (int)std::min<size_t>(per, v.size() - s0);
                    Proto q;
                    q.it = Item{0, (int32_t)deg, (uint8_t)nb, (uint8_t)lg, (uint8_t)ITEM_LANE, (uint8_t)pr};
                    q.g0 = (int64_t)gb.size();
                    for (int l = 0; l < nb; ++l) gb.push_back(v[s0 + l]);
                    kinds[0].push_back(q);
                    if (lg == 0) ++L.n_lane;
                    else ++L.n_seg;
                }
            }
    for (auto& kv : wgb) {
        const int64_t i = kv.second;
        Proto q;
        q.it = Item{0, (int32_t)(d->block_off[i + 1] - d->block_off[i]), 1, 0, (uint8_t)ITEM_WG, d->block_proj[i]};
        q.g0 = (int64_t)gb.size();
        gb.push_back(i);
        kinds[1].push_back(q);
    }
    L.n_wg = (int64_t)kinds[1].size();

    // deal: chunk c takes items c, c + nchunks, ... of each kind (WG items:
    // item r nchunks + c in even rounds r, r nchunks + nchunks - 1 - c in odd
    // ones); stream positions follow the final item order
    L.chunks.assign((size_t)nchunks, Chunk{});
    std::vector<int64_t> g0s;
    int64_t pos = 0;
    for (int k = 0; k < 2; ++k) {
        const auto& v = kinds[k];
        for (int c = 0; c < nchunks; ++c) {
            int32_t* r = k == 0 ? &L.chunks[c].a0 : &L.chunks[c].b0;
            r[0] = (int32_t)L.items.size();
            for (size_t r0 = 0; r0 < v.size(); r0 += (size_t)nchunks) {
                const bool back = k == 1 && (r0 / (size_t)nchunks) % 2 == 1;
                const size_t q = r0 + (back ? (size_t)(nchunks - 1 - c) : (size_t)c);
                if (q >= v.size()) continue;
                Item it = v[q].it;
                it.base = pos;
                pos += (int64_t)it.d * it.nb;
                L.items.push_back(it);
                g0s.push_back(v[q].g0);
            }
            r[1] = (int32_t)L.items.size();
        }
    }
    // waves' shares of each chunk's lane items.  With few classes (kernel
    // paths: lanes per block, register rows, projection) a wave takes every
    // kWaves-th item (w[0] = -1): the shares balance by themselves and each
    // wave meets every class once.  With many classes a wave takes a
    // contiguous share, split at equal estimated cost (rows of the group's
    // register class, plus a fixed part), so that it meets only a few classes
    // (each class change restarts the wave's prefetch pipeline).
    auto item_class = [&](const Item& it) -> int {
        const int64_t R = ((int64_t)it.d + (1 << it.lg) - 1) >> it.lg;
        const int rows = it.lg == 0 ? (it.d <= 4 ? 4 : it.d <= 8 ? 8 : it.d <= 12 ? 12 : it.d <= 16 ? 16
                                                                                     : it.d <= 24 ? 24 : 32)
                                    : (R <= 8 ? 8 : pmax);
        return (it.lg * 64 + rows) * 4 + it.proj;
    };
    std::vector<int> classes;
    for (const Item& it : L.items)
        if (it.kind == ITEM_LANE) classes.push_back(item_class(it));
    std::sort(classes.begin(), classes.end());
    const bool strided = std::unique(classes.begin(), classes.end()) - classes.begin() <= kStridedClasses;
    auto item_cost = [&](const Item& it) -> int64_t {
        int64_t rows;
        if (it.lg == 0) rows = it.d <= 4 ? 4 : it.d <= 8 ? 8 : it.d <= 12 ? 12 : it.d <= 16 ? 16 : it.d <= 24 ? 24 : 32;
        else rows = (((int64_t)it.d + (1 << it.lg) - 1) >> it.lg) <= 8 ? 8 : pmax;
        return rows + 4;
    };
    for (int c = 0; c < nchunks && strided; ++c) {
        Chunk& ch = L.chunks[c];
        for (int q = 0; q <= kWaves; ++q) ch.w[q] = -1;
    }
    for (int c = 0; c < nchunks && !strided; ++c) {
        Chunk& ch = L.chunks[c];
        int64_t tot = 0;
        for (int32_t q = ch.a0; q < ch.a1; ++q) tot += item_cost(L.items[q]);
        int64_t acc = 0;
        int wv = 1;
        ch.w[0] = ch.a0;
        for (int32_t q = ch.a0; q < ch.a1 && wv < kWaves; ++q) {
            acc += item_cost(L.items[q]);
            while (wv < kWaves && acc * kWaves >= tot * wv) ch.w[wv++] = q + 1;
        }
        while (wv < kWaves) ch.w[wv++] = ch.a1;
        ch.w[kWaves] = ch.a1;
    }

    // stream position -> original column: edge e = k S + s of block b of a
    // LANE group sits at base + k nb S + b S + s for k < R - 1, and the last
    // row is compacted: base + (R - 1) nb S + b rem + s
    L.src.assign((size_t)pos, 0);
    const int64_t nit = (int64_t)L.items.size();
    parallel_for(nit, 4096, [&](int64_t lo, int64_t hi) {
        for (int64_t q = lo; q < hi; ++q) {
            const Item& it = L.items[q];
            const int64_t g0 = g0s[q];
            if (it.kind == ITEM_LANE) {
                const int64_t S = (int64_t)1 << it.lg, nb = it.nb, deg = it.d;
                const int64_t R = (deg + S - 1) / S, rem = deg - (R - 1) * S, W = nb * S;
                for (int64_t l = 0; l < nb; ++l) {
                    const int64_t c0 = d->block_off[gb[g0 + l]];
                    for (int64_t e = 0; e < deg; ++e) {
                        const int64_t k = e / S, s = e % S;
                        const int64_t off = k < R - 1 ? k * W + l * S + s : (R - 1) * W + l * rem + s;
                        L.src[it.base + off] = c0 + e;
                    }
                }
            } else {
                const int64_t c0 = d->block_off[gb[g0]];
                for (int k = 0; k < it.d; ++k) L.src[it.base + k] = c0 + k;
            }
        }
    });
}

static int device_cus(int dev)
{
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    return v;
}

static size_t device_max_lds(int dev)
{
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        v = 65536;
    return (size_t)v;
}

template <typename T>
static dl_status dalloc(dl_problem* p, T** ptr, size_t count, const char* what)
{
    *ptr = nullptr;
    if (count == 0) count = 1;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of %zu bytes for %s failed: %s", count * sizeof(T), what, hipGetErrorString(e));
        return DL_ERR_OUT_OF_MEMORY;
    }
    p->allocs.push_back(q);
    p->device_bytes += count * sizeof(T);
    *ptr = (T*)q;
    return DL_OK;
}

static void free_problem(dl_problem* p)
{
    if (!p) return;
    if (p->gc.exec) (void)hipGraphExecDestroy(p->gc.exec);
    if (p->gc.graph) (void)hipGraphDestroy(p->gc.graph);
    for (auto e : p->gc.ev)
        if (e) (void)hipEventDestroy(e);
    for (void* q : p->allocs) (void)hipFree(q);
    if (p->st_host) (void)hipHostFree(p->st_host);
    delete p;
}

// Work layout of a problem: largest one-lane degree and rows per lane (each
// clamped to the kernel variant's register budget) and workgroups per CU.
struct LayoutChoice {
    // wg_min: blocks of at least this many edges (beyond the one-lane ones)
    // are WG items; 0: only those too long for 64-lane segments
    int lane_cap = 1 << 30, seg_rmax = 1 << 30, chunk_mult = 1, wg_min = 0, tuned = 0;
};

static dl_status tune_layout(const dl_problem_desc* d, const dl_problem_opts& opts, hipStream_t s,
                             LayoutChoice* out);

// |A'|^2 = largest eigenvalue of A'A'^T, A' = D A D_v^{-1} (entries of column e
// in planes f < count[e] of crow/cval, D in original row order, v2 = v^2 or
// empty), by power iteration: z <- A'(A'^T z) / |.| from z = 1 until the
// Rayleigh quotient changes by less than 1e-10 (at most 500 steps).  The
// quotient approaches the eigenvalue from below; the result is raised by
// 1e-3 so that a step of 1/L stays on the safe side.
static double power_anorm2(int64_t m, int64_t n, int nf, const std::vector<int32_t>& crow,
                           const std::vector<double>& cval, const std::vector<uint8_t>& count,
                           const std::vector<double>& D, const std::vector<double>& v2)
{
    auto coef = [&](int f, int64_t e) {
        const double a = cval[(size_t)f * n + e] * D[crow[(size_t)f * n + e]];
        return v2.empty() ? a : a / std::sqrt(v2[e]);
    };
    std::vector<double> z((size_t)m, 1.0), y((size_t)n, 0.0), z2((size_t)m, 0.0);
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(16, n / (1 << 16)));
    std::vector<std::vector<double>> part((size_t)nt, std::vector<double>((size_t)m, 0.0));
    double lam = 0.0;
    for (int it = 0; it < 500; ++it) {
        parallel_for(n, 1 << 16, [&](int64_t lo, int64_t hi) {
            for (int64_t e = lo; e < hi; ++e) {
                double acc = 0.0;
                for (int f = 0; f < count[e]; ++f) acc += coef(f, e) * z[crow[(size_t)f * n + e]];
                y[e] = acc;
            }
        });
        std::vector<std::thread> th;
        for (int t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                std::vector<double>& pz = part[t];
                std::fill(pz.begin(), pz.end(), 0.0);
                const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
                for (int64_t e = lo; e < hi; ++e)
                    for (int f = 0; f < count[e]; ++f) pz[crow[(size_t)f * n + e]] += coef(f, e) * y[e];
            });
        for (auto& x : th) x.join();
        double zz = 0.0, zm = 0.0;
        for (int64_t r = 0; r < m; ++r) {
            double a = 0.0;
            for (int t = 0; t < nt; ++t) a += part[t][r];
            z2[r] = a;
            zz += z[r] * z[r];
            zm += z[r] * a;
        }
        const double q = zz > 0.0 ? zm / zz : 0.0;
        double nz = 0.0;
        for (int64_t r = 0; r < m; ++r) nz += z2[r] * z2[r];
        nz = std::sqrt(nz);
        if (!(nz > 0.0)) break;
        for (int64_t r = 0; r < m; ++r) z[r] = z2[r] / nz;
        const bool done = it > 0 && std::fabs(q - lam) <= 1e-10 * q;
        lam = q;
        if (done) break;
    }
    return lam > 0.0 ? lam * (1.0 + 1e-3) : 1.0;
}

// builds and uploads a validated problem with the given layout
static dl_status create_with(const dl_problem_desc* d, const dl_problem_opts& opts, int solve_ok,
                             const LayoutChoice& lc, hipStream_t s, dl_problem** out, int col_entries = 1)
{
    dl_status st = DL_OK;
    const int64_t m = d->m, n = d->n;
    dl_problem* p = new dl_problem();
    {
        const hipError_t e = hipGetDevice(&p->device);
        if (e != hipSuccess) { delete p; return hip_fail(e, "hipGetDevice"); }
    }
    p->m = m;
    p->n = n;
    p->nblocks = d->num_blocks;
    p->storage = opts.storage;
    p->solve_ok = solve_ok;
    p->det = opts.deterministic;
    p->J = (int)m;

    // per column: rows and values of its entries, entry f in plane f
    // (crow[f n + e]); an empty column and missing entries: row 0, a = 0
    const int nf = std::max(1, col_entries);
    p->nf = nf;
    std::vector<int32_t> crow((size_t)n * nf, 0);
    std::vector<double> cval((size_t)n * nf, 0.0);
    std::vector<uint8_t> ccount(nf > 1 ? (size_t)n : 0, 0);
    if (d->layout == DL_CSC) {
        for (int64_t e = 0; e < n; ++e) {
            const int64_t lo = d->ptr ? d->ptr[e] : e, hi = d->ptr ? d->ptr[e + 1] : e + 1;
            for (int64_t k = lo; k < hi; ++k) {
                crow[(size_t)(k - lo) * n + e] = d->idx[k];
                cval[(size_t)(k - lo) * n + e] = d->val[k];
            }
            if (nf > 1) ccount[e] = (uint8_t)(hi - lo);
        }
    } else {
        std::vector<uint8_t> cnt((size_t)n, 0);
        for (int64_t j = 0; j < m; ++j)
            for (int64_t k = d->ptr[j]; k < d->ptr[j + 1]; ++k) {
                const int32_t e = d->idx[k];
                const size_t f = cnt[e]++;
                crow[f * n + e] = (int32_t)j;
                cval[f * n + e] = d->val[k];
            }
        if (nf > 1) ccount = cnt;
    }
    // primal scale v (regularizer gamma/2 v^2 x^2) and Jacobi row scale of A D_v^{-1}
    std::vector<double> v2;
    if (opts.primal_scale != 0) {
        v2.resize((size_t)n);
        for (int64_t e = 0; e < n; ++e) {
            double v = opts.v ? opts.v[e] : 0.0;
            if (opts.primal_scale == 1) {
                // column norm |A_{:,e}|_2 over the column's entries
                double c2 = 0.0;
                for (int f = 0; f < nf; ++f) c2 += cval[(size_t)f * n + e] * cval[(size_t)f * n + e];
                v = std::sqrt(c2);
            }
            if (!(v > 0.0)) v = 1.0;
            v2[e] = v * v;
        }
        p->has_w = 1;
    }
    std::vector<double> r2((size_t)m, 0.0);
    std::vector<int64_t> rdeg((size_t)m, 0);
    for (int64_t e = 0; e < n; ++e) {
        const double z = cval[e];
        r2[crow[e]] += p->has_w ? z * z / v2[e] : z * z;
        rdeg[crow[e]] += 1;
        for (int f = 1; f < nf && f < ccount[e]; ++f) {
            const double zf = cval[(size_t)f * n + e];
            const int32_t rf = crow[(size_t)f * n + e];
            r2[rf] += p->has_w ? zf * zf / v2[e] : zf * zf;
            rdeg[rf] += 1;
        }
    }
    // a plane whose entry is present in every column with one row (a dense
    // row such as the count row): its sums are combined per wave in the
    // multi-entry kernel instead of one LDS atomic per active edge
    for (int f = 0; f < nf && nf > 1 && p->dense_f < 0 && n > 0; ++f) {
        bool same = true;
        for (int64_t e = 0; e < n && same; ++e)
            same = ccount[e] > f && crow[(size_t)f * n + e] == crow[(size_t)f * n];
        if (same) p->dense_f = f;
    }
    // relabel rows by descending degree (ties by index): hot rows first
    std::vector<int32_t> orig((size_t)m), newid((size_t)m);
    std::iota(orig.begin(), orig.end(), 0);
    std::stable_sort(orig.begin(), orig.end(), [&](int32_t a, int32_t b) { return rdeg[a] > rdeg[b]; });
    for (int64_t j = 0; j < m; ++j) newid[orig[j]] = (int32_t)j;
    if (p->dense_f >= 0) p->dense_row = newid[crow[(size_t)p->dense_f * n]];
    std::vector<double> bD((size_t)m), Dv((size_t)m);
    for (int64_t j = 0; j < m; ++j) {
        const int32_t o = orig[j];
        bD[j] = d->b[o];
        Dv[j] = (opts.row_normalize && r2[o] > 0.0) ? 1.0 / std::sqrt(r2[o]) : 1.0;
    }
    // one family: A D_v^{-1} has orthogonal rows, so |A'|^2 is the largest
    // squared row norm (1 after row normalization, empty rows aside);
    // several entries per column: power iteration on A'A'^T
    if (nf > 1) {
        std::vector<double> Do((size_t)m);
        for (int64_t j = 0; j < m; ++j) Do[orig[j]] = Dv[j];
        p->anorm2 = power_anorm2(m, n, nf, crow, cval, ccount, Do, v2);
    } else {
        double mx = 0.0;
        for (int64_t j = 0; j < m; ++j) mx = std::max(mx, opts.row_normalize ? (r2[j] > 0.0 ? 1.0 : 0.0) : r2[j]);
        p->anorm2 = mx > 0.0 ? mx : 1.0;
    }
    // per-edge bounds are stored when any block has them (box and capped)
    for (int64_t i = 0; i < d->num_blocks && !p->has_box; ++i) p->has_box = d->block_proj[i] != DL_PROJ_SIMPLEX;
    for (int64_t i = 0; i < d->num_blocks && !p->has_cut; ++i) p->has_cut = d->block_proj[i] == DL_PROJ_CAPPED;

    // work items and chunks
    const int cus = device_cus(p->device);
    int nch = (int)std::min<int64_t>((int64_t)cus * lc.chunk_mult, std::max<int64_t>(1, (n + 32767) / 32768));
    HostLayout L;
    const size_t max_lds = device_max_lds(p->device);
    // bytes of one LDS sum in gap-check passes: f32, or a 64-bit integer in
    // deterministic mode.  Ordinary passes hold lam and the a x sum per row:
    // 8 bytes (FP64) when every row fits at 16 bytes, else f32 for the K rows
    // that fit at 12 (deterministic mode: the 64-bit integer, 16 bytes).
    // Problems with more rows than fit at 16 bytes but no more than fit at
    // 12 keep the 16-byte capacity and their coldest rows beyond it.
    const int64_t hes = p->det ? 8 : 4, lds_free = (int64_t)max_lds - 4 * kWaves * (int64_t)sizeof(double);
    // (the multi-entry kernel keeps FP64 sums for every row in LDS)
    const int64_t kwide = lds_free / 16, knarrow = (p->det || nf > 1) ? kwide : lds_free / 12;
    int64_t kmax = m <= kwide ? m : (m > knarrow ? knarrow : kwide);
    p->K = (int)std::max<int64_t>(0, std::min<int64_t>(m, kmax));
    const bool f64 = opts.storage == DL_F64, tail = p->K < m;
    // check passes: without tail rows the c x and v^2 x^2 sums of the first
    // Kc rows join lam and the a x sums in LDS; with tail rows lam is read
    // from memory and the c x and v^2 x^2 sums of the first Kc rows join the
    // a x sums (all K rows with f32 sums)
    const int64_t kc = tail ? (lds_free - (int64_t)p->K * hes) / (2 * hes)
                            : (lds_free - (int64_t)p->K * (8 + hes)) / (2 * hes);
    p->Kc = (int)std::max<int64_t>(0, std::min<int64_t>(p->K, kc));
    p->lane_cap = std::min(lc.lane_cap, lane_cap(f64, p->has_w != 0, tail));
    p->seg_rmax = std::min(lc.seg_rmax, seg_rmax(f64, p->has_w != 0, tail));
    if (nf > 1) {
        // multi-entry columns: no per-row c x, v^2 x^2 sums (the gap's
        // restoration is a pass of its own) and smaller lane classes
        p->Kc = 0;
        p->lane_cap = std::min(p->lane_cap, kMfLaneCap);
        p->seg_rmax = std::min(p->seg_rmax, kMfRmax);
    }
    p->chunk_mult = lc.chunk_mult;
    p->tuned = lc.tuned;
    // a threshold beyond what 64-lane segments hold changes nothing
    p->wg_min = lc.wg_min > 0 && lc.wg_min <= 64 * p->seg_rmax ? std::max(lc.wg_min, p->lane_cap + 1) : 0;
    // the kernel variant's largest row class; segments of 4, 16 or 64 lanes
    // only for the kernels of problems with capped blocks or in
    // deterministic mode; the multi-entry kernel also has a 4-row class
    const int pmax = nf > 1 ? kMfRmax : seg_rmax(f64, p->has_w != 0, tail);
    build_items(d, nch, p->lane_cap, p->seg_rmax, pmax, nf == 1 && (p->has_cut || p->det), p->wg_min, nf > 1, L);
    p->nchunks = nch;
    p->nitems = (int)L.items.size();
    p->n_lane = L.n_lane;
    p->n_seg = L.n_seg;
    p->n_wg = L.n_wg;
    p->nblk2 = (p->J + 63) / 64;

    // stream arrays
    const size_t es = opts.storage == DL_F64 ? 8 : (opts.storage == DL_F32 ? 4 : 2);
    std::vector<unsigned char> Ah((size_t)n * es), Ch((size_t)n * es);
    std::vector<int32_t> dsth((size_t)n);
    // planes 1..nf-1 of multi-entry columns (coefficients, internal rows)
    std::vector<unsigned char> A2h((size_t)(nf - 1) * n * es);
    std::vector<int32_t> dst2h((size_t)(nf - 1) * n);
    std::vector<float> Uh(p->has_box ? (size_t)n : 0), IVh(p->has_w ? (size_t)n : 0);
    int64_t box_edges = 0;
    {
        std::vector<uint8_t> ebox;
        if (p->has_box) {
            ebox.assign((size_t)n, 0);
            for (int64_t i = 0; i < d->num_blocks; ++i)
                if (d->block_proj[i] != DL_PROJ_SIMPLEX)
                    for (int64_t e = d->block_off[i]; e < d->block_off[i + 1]; ++e) ebox[e] = 1;
        }
        parallel_for(n, 1 << 20, [&](int64_t lo, int64_t hi) {
            for (int64_t q = lo; q < hi; ++q) {
                const int64_t e = L.src[q];
                const double a = cval[e], c = d->c[e];
                if (opts.storage == DL_F64) { ((double*)Ah.data())[q] = a; ((double*)Ch.data())[q] = c; }
                else if (opts.storage == DL_F32) { ((float*)Ah.data())[q] = (float)a; ((float*)Ch.data())[q] = (float)c; }
                else { ((uint16_t*)Ah.data())[q] = to_bf16(a); ((uint16_t*)Ch.data())[q] = to_bf16(c); }
                dsth[q] = newid[crow[e]];
                for (int f = 1; f < nf; ++f) {
                    const size_t qf = (size_t)(f - 1) * n + q;
                    const double af = cval[(size_t)f * n + e];
                    if (opts.storage == DL_F64) ((double*)A2h.data())[qf] = af;
                    else if (opts.storage == DL_F32) ((float*)A2h.data())[qf] = (float)af;
                    else ((uint16_t*)A2h.data())[qf] = to_bf16(af);
                    dst2h[qf] = newid[crow[(size_t)f * n + e]];
                }
                if (p->has_box) Uh[q] = (float)(d->upper ? d->upper[e] : 1.0);
                if (p->has_w) IVh[q] = (float)(1.0 / v2[e]);
            }
        });
        if (p->has_box)
            for (int64_t e = 0; e < n; ++e) box_edges += ebox[e];
    }
    p->stream_bytes = n * (int64_t)(es + nf * (es + 4)) + (p->has_box ? 4 * box_edges : 0) + (p->has_w ? 4 * n : 0);
    if (p->det) {
        // fixed-point scales of the three per-destination sums: 2^F with F
        // the largest integer such that a bound on any row's sum (and so on
        // any partial of it) stays below 2^60 (x_e <= 1 on simplex and capped
        // blocks, <= u_e on box blocks)
        std::vector<double> bnd(3 * (size_t)m, 0.0);
        for (int64_t i = 0; i < d->num_blocks; ++i) {
            const int pr = d->block_proj[i];
            for (int64_t e = d->block_off[i]; e < d->block_off[i + 1]; ++e) {
                const double ue = d->upper ? d->upper[e] : 1.0;
                const double xm = pr == DL_PROJ_SIMPLEX ? 1.0 : (pr == DL_PROJ_BOX ? ue : std::min(ue, 1.0));
                const size_t j = (size_t)crow[e];
                bnd[j] += std::fabs(cval[e]) * xm;
                bnd[m + j] += std::fabs(d->c[e]) * xm;
                bnd[2 * m + j] += (p->has_w ? v2[e] : 1.0) * xm * xm;
            }
        }
        for (int q = 0; q < 3; ++q) {
            double b = 0.0;
            for (int64_t j = 0; j < m; ++j) b = std::max(b, bnd[(size_t)q * m + j]);
            b = b > 0.0 ? b * 1.01 : 1.0;
            const int F = (int)std::floor(60.0 - std::log2(b));
            p->qs[q] = std::ldexp(1.0, F);
        }
    }

    // device allocation and upload
#define ALLOC(ptr, count, what)                                      \
    do {                                                             \
        st = dalloc(p, &(ptr), (count), what);                       \
        if (st != DL_OK) { free_problem(p); return st; }             \
    } while (0)
#define UP(dstp, srcp, bytes, what)                                                          \
    do {                                                                                     \
        hipError_t e_ = hipMemcpyAsync((dstp), (srcp), (bytes), hipMemcpyHostToDevice, s);   \
        if (e_ != hipSuccess) { st = hip_fail(e_, what); free_problem(p); return st; }       \
    } while (0)
    unsigned char *Ad, *Cd;
    ALLOC(Ad, (size_t)n * es, "a");
    ALLOC(Cd, (size_t)n * es, "c");
    p->A = Ad;
    p->C = Cd;
    ALLOC(p->dst, (size_t)n, "dst");
    if (p->has_box) ALLOC(p->U, (size_t)n, "upper");
    if (p->has_w) ALLOC(p->IV, (size_t)n, "primal scale");
    ALLOC(p->perm, (size_t)n, "perm");
    ALLOC(p->items, L.items.size(), "items");
    ALLOC(p->chunks, L.chunks.size(), "chunks");
    ALLOC(p->b, (size_t)m, "b");
    ALLOC(p->D, (size_t)m, "D");
    ALLOC(p->orig, (size_t)m, "orig");
    // partial sums: f32, or 64-bit integers (two f32 slots) in deterministic mode
    ALLOC(p->part, (size_t)3 * nch * std::max(1, p->K) * (p->det ? 2 : 1), "partials");
    ALLOC(p->tail, (size_t)3 * m, "tail");
    ALLOC(p->obj_part, (size_t)3 * nch, "objective partials");
    ALLOC(p->blockpart, (size_t)p->nblk2 * kRedStride, "block partials");
    ALLOC(p->lam_int, (size_t)m, "lambda");
    ALLOC(p->eval6, 8, "eval");
    if (nf > 1) {
        for (int f = 1; f < nf; ++f) {
            unsigned char* Af;
            ALLOC(Af, (size_t)n * es, "coefficient plane");
            p->A2[f - 1] = Af;
            ALLOC(p->dst2[f - 1], (size_t)n, "row plane");
        }
        ALLOC(p->srow, (size_t)m, "row ratios");
        ALLOC(p->corr_part, (size_t)nch, "restoration partials");
    }
    ALLOC(p->lam, (size_t)m, "lam");
    ALLOC(p->y, (size_t)m, "y");
    ALLOC(p->yp, (size_t)m, "y_prev");
    ALLOC(p->G, (size_t)m, "G");
    ALLOC(p->Gp, (size_t)m, "G_prev");
    ALLOC(p->lam_eval, (size_t)m, "lam_eval");
    ALLOC(p->st, 1, "state");
    UP(p->A, Ah.data(), Ah.size(), "upload a");
    UP(p->C, Ch.data(), Ch.size(), "upload c");
    UP(p->dst, dsth.data(), dsth.size() * 4, "upload dst");
    for (int f = 1; f < nf; ++f) {
        UP(p->A2[f - 1], A2h.data() + (size_t)(f - 1) * n * es, (size_t)n * es, "upload plane");
        UP(p->dst2[f - 1], dst2h.data() + (size_t)(f - 1) * n, (size_t)n * 4, "upload plane rows");
    }
    if (p->has_box) UP(p->U, Uh.data(), Uh.size() * 4, "upload upper");
    if (p->has_w) UP(p->IV, IVh.data(), IVh.size() * 4, "upload scale");
    UP(p->perm, L.src.data(), L.src.size() * 8, "upload perm");
    UP(p->items, L.items.data(), L.items.size() * sizeof(Item), "upload items");
    UP(p->chunks, L.chunks.data(), L.chunks.size() * sizeof(Chunk), "upload chunks");
    UP(p->b, bD.data(), (size_t)m * 8, "upload b");
    UP(p->D, Dv.data(), (size_t)m * 8, "upload D");
    UP(p->orig, orig.data(), (size_t)m * 4, "upload orig");
    {
        hipError_t e = hipMemsetAsync(p->tail, 0, (size_t)3 * m * sizeof(double), s);
        if (e != hipSuccess) { st = hip_fail(e, "clear tail"); free_problem(p); return st; }
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) { st = hip_fail(e, "upload"); free_problem(p); return st; }
        e = hipHostMalloc((void**)&p->st_host, 2 * sizeof(SolveState), hipHostMallocDefault);
        if (e != hipSuccess) { p->st_host = nullptr; st = hip_fail(e, "pinned state"); free_problem(p); return st; }
        e = dlh::ensure_grad_attributes(p->device);
        if (e != hipSuccess) { st = hip_fail(e, "kernel LDS attribute"); free_problem(p); return st; }
    }
#undef ALLOC
#undef UP
    *out = p;
    return DL_OK;
}

// Autotune: every k-th block of the problem (about kTuneNnz nonzeros, all m
// destinations, same projection types and scales, capacities scaled by the
// sampled fraction of nonzeros so that they bind as often as in the whole
// problem) is solved for kTunePrices iterations at gamma = kTuneGamma with
// natural steps; the gradient kernel is then timed at those prices for each
// layout on a coordinate search (one parameter at a time, the others at the
// best so far; a change is kept when it is at least kTuneGain faster).  The
// kernel's cost depends on the prices through the projections' active sets,
// so prices of zero (every block unconstrained by capacity) would time a
// different mix of threshold loops than the solver runs.
constexpr int64_t kTuneNnz = (int64_t)16 << 20;
constexpr int kTunePrices = 200;
constexpr double kTuneGamma = 1e-3;
constexpr double kTuneGain = 0.01;

static dl_status tune_layout(const dl_problem_desc* d, const dl_problem_opts& opts, hipStream_t s,
                             LayoutChoice* out)
{
    const int64_t I = d->num_blocks, n = d->n;
    const int64_t step = std::max<int64_t>(1, (n + kTuneNnz - 1) / kTuneNnz);
    // sample columns, one CSC entry each
    std::vector<int32_t> crow((size_t)n, 0);
    std::vector<double> cval((size_t)n, 0.0);
    if (d->layout == DL_CSC) {
        for (int64_t e = 0; e < n; ++e) {
            const int64_t lo = d->ptr ? d->ptr[e] : e, hi = d->ptr ? d->ptr[e + 1] : e + 1;
            if (hi > lo) { crow[e] = d->idx[lo]; cval[e] = d->val[lo]; }
        }
    } else {
        for (int64_t j = 0; j < d->m; ++j)
            for (int64_t k = d->ptr[j]; k < d->ptr[j + 1]; ++k) { crow[d->idx[k]] = (int32_t)j; cval[d->idx[k]] = d->val[k]; }
    }
    std::vector<int64_t> off(1, 0);
    std::vector<uint8_t> proj;
    std::vector<int32_t> idx;
    std::vector<double> val, c, up, v;
    for (int64_t i = 0; i < I; i += step) {
        for (int64_t e = d->block_off[i]; e < d->block_off[i + 1]; ++e) {
            idx.push_back(crow[e]);
            val.push_back(cval[e]);
            c.push_back(d->c[e]);
            if (d->upper) up.push_back(d->upper[e]);
            if (opts.primal_scale == 2) v.push_back(opts.v[e]);
        }
        off.push_back((int64_t)idx.size());
        proj.push_back(d->block_proj[i]);
    }
    const double frac = n > 0 ? (double)idx.size() / (double)n : 1.0;
    std::vector<double> bs((size_t)d->m);
    for (int64_t j = 0; j < d->m; ++j) bs[j] = d->b[j] * frac;
    dl_problem_desc sd = *d;
    sd.n = sd.nnz = (int64_t)idx.size();
    sd.layout = DL_CSC;
    sd.ptr = nullptr;
    sd.idx = idx.data();
    sd.val = val.data();
    sd.c = c.data();
    sd.b = bs.data();
    sd.num_blocks = (int64_t)proj.size();
    sd.block_off = off.data();
    sd.block_proj = proj.data();
    sd.upper = d->upper ? up.data() : nullptr;
    dl_problem_opts so = opts;
    so.autotune = 0;
    so.v = opts.primal_scale == 2 ? v.data() : nullptr;
    int sample_solve_ok = 1, ce = 1;
    dl_status st = validate_impl(&sd, &so, &sample_solve_ok, &ce);
    if (st != DL_OK) return st;

    double* lam = nullptr;
    HIP_TRY(hipMalloc(&lam, (size_t)d->m * sizeof(double)), "tuning buffer");
    {
        const hipError_t e = hipMemsetAsync(lam, 0, (size_t)d->m * sizeof(double), s);
        if (e != hipSuccess) st = hip_fail(e, "tuning buffer");
    }

    // timed layouts by their effective (lane_cap, seg_rmax, wg_min, chunk_mult)
    std::vector<std::pair<std::array<int, 4>, double>> timed;
    bool prices = false;
    auto time_layout = [&](const LayoutChoice& lc, double* ms_out) -> dl_status {
        dl_problem* sp = nullptr;
        dl_status r = create_with(&sd, so, sample_solve_ok, lc, s, &sp);
        if (r != DL_OK) return r;
        if (!prices) {
            // representative prices from the first layout built (a solve's
            // iterates do not depend on the layout beyond rounding order)
            prices = true;
            if (sample_solve_ok) {
                dl_solve_opts o;
                dl_solve_opts_init(&o);
                o.gamma0 = o.gamma_final = kTuneGamma;
                o.max_iters = kTunePrices;
                o.tol_rel_gap = -1.0;
                o.preset = DL_PRESET_NATURAL;
                dl_solve_result res;
                const dl_status rs = dl_solve(sp, &o, lam, &res, s);
                if (rs != DL_OK && rs != DL_ERR_NOT_CONVERGED) {
                    // no usable prices (a non-finite objective): time at zero
                    const hipError_t e = hipMemsetAsync(lam, 0, (size_t)d->m * sizeof(double), s);
                    if (e != hipSuccess) r = hip_fail(e, "tuning buffer");
                }
            }
        }
        const std::array<int, 4> key{sp->lane_cap, sp->seg_rmax, sp->wg_min, sp->chunk_mult};
        for (auto& kv : timed)
            if (kv.first == key) {
                *ms_out = kv.second;
                dl_problem_destroy(sp);
                return r;
            }
        std::vector<double> t;
        double ms = 0.0;
        if (r == DL_OK) r = dl_time_grad_kernel(sp, lam, kTuneGamma, 4, 0, &ms, s);
        for (int q = 0; q < 5 && r == DL_OK; ++q) {
            r = dl_time_grad_kernel(sp, lam, kTuneGamma, 4, 0, &ms, s);
            t.push_back(ms);
        }
        dl_problem_destroy(sp);
        if (r != DL_OK) return r;
        std::sort(t.begin(), t.end());
        *ms_out = t[t.size() / 2];
        timed.push_back({key, *ms_out});
        return DL_OK;
    };

    LayoutChoice best = *out;   // the caller's layout (defaults where unset)
    best.tuned = 1;
    double best_ms = INFINITY;
    if (st == DL_OK) st = time_layout(best, &best_ms);
    // coordinate search: largest one-lane block, rows per lane, smallest
    // workgroup block, workgroups per CU
    const int lcaps[] = {24, 16, 8};
    const int rmaxs[] = {12, 8, 4};
    const int wgmins[] = {2048, 1024, 512, 256};
    const int mults[] = {2};
    for (int axis = 0; axis < 4 && st == DL_OK; ++axis) {
        const int* vals = axis == 0 ? lcaps : axis == 1 ? rmaxs : axis == 2 ? wgmins : mults;
        const int nv = axis == 0 ? 3 : axis == 1 ? 3 : axis == 2 ? 4 : 1;
        LayoutChoice axis_best = best;
        double axis_ms = best_ms;
        for (int q = 0; q < nv && st == DL_OK; ++q) {
            LayoutChoice cand = best;
            int& slot = axis == 0 ? cand.lane_cap : axis == 1 ? cand.seg_rmax : axis == 2 ? cand.wg_min : cand.chunk_mult;
            slot = vals[q];
            double ms = 0.0;
            st = time_layout(cand, &ms);
            if (st == DL_OK && ms < axis_ms) {
                axis_ms = ms;
                axis_best = cand;
            }
        }
        if (axis_ms < best_ms * (1.0 - kTuneGain)) {
            best = axis_best;
            best_ms = axis_ms;
        }
    }
    (void)hipFree(lam);
    if (st == DL_OK) *out = best;
    return st;
}

extern "C" dl_status dl_problem_create(const dl_problem_desc* d, const dl_problem_opts* opts_in,
                                       void* hip_stream, dl_problem** out)
{
    if (!out) { set_error("out is NULL"); return DL_ERR_INVALID_ARG; }
    *out = nullptr;
    dl_problem_opts opts;
    dl_problem_opts_init(&opts);
    if (opts_in) opts = *opts_in;
    if (opts.autotune != 0 && opts.autotune != 1) { set_error("autotune must be 0 or 1"); return DL_ERR_INVALID_ARG; }
    int solve_ok = 1, col_entries = 1;
    dl_status st = validate_impl(d, &opts, &solve_ok, &col_entries);
    if (st != DL_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    LayoutChoice lc;
    if (opts.lane_cap > 0) lc.lane_cap = opts.lane_cap;
    if (opts.seg_rmax > 0) lc.seg_rmax = opts.seg_rmax;
    if (opts.wg_min > 0) lc.wg_min = opts.wg_min;
    if (opts.chunks_per_cu > 0) lc.chunk_mult = opts.chunks_per_cu;
    // (multi-entry columns keep the default layout: the tuner samples one
    // entry per column)
    if (opts.autotune && col_entries <= 1) {
        st = tune_layout(d, opts, s, &lc);
        if (st != DL_OK) return st;
    }
    return create_with(d, opts, solve_ok, lc, s, out, col_entries);
}

extern "C" dl_status dl_problem_destroy(dl_problem* p)
{
    if (!p) return DL_OK;
    (void)hipDeviceSynchronize();
    free_problem(p);
    return DL_OK;
}

namespace dlh {
// The gradient kernels' dynamic-LDS limit is a process-wide attribute of each
// kernel.  It is raised once per device to the device's whole LDS (every
// problem's need fits under it) and never lowered, under a lock, so problems
// created concurrently (the server's loader threads) cannot shrink it below
// what a running launch uses.
hipError_t ensure_grad_attributes(int device)
{
    static std::mutex mu;
    static std::vector<int> done;
    std::lock_guard<std::mutex> lk(mu);
    if (std::find(done.begin(), done.end(), device) != done.end()) return hipSuccess;
    const hipError_t e = set_grad_attributes(device_max_lds(device));
    if (e == hipSuccess) done.push_back(device);
    return e;
}

void destroy_idle(dl_problem* p)
{
    if (p) free_problem(p);
}
}  // namespace dlh

extern "C" dl_status dl_problem_get_info(const dl_problem* p, dl_problem_info* info)
{
    if (!p || !info) { set_error("NULL argument"); return DL_ERR_INVALID_ARG; }
    info->m = p->m;
    info->n = p->n;
    info->num_blocks = p->nblocks;
    info->lane_groups = p->n_lane;
    info->seg_groups = p->n_seg;
    info->wg_blocks = p->n_wg;
    info->chunks = p->nchunks;
    info->lds_rows = p->K;
    info->stream_bytes = p->stream_bytes;
    info->device_bytes = (int64_t)p->device_bytes;
    info->storage = p->storage;
    info->has_box = p->has_box;
    info->deterministic = p->det;
    info->has_capped = p->has_cut;
    info->col_entries = p->nf;
    info->wg_min = p->wg_min;
    info->lane_cap = p->lane_cap;
    info->seg_rmax = p->seg_rmax;
    info->chunks_per_cu = p->chunk_mult;
    info->tuned = p->tuned;
    info->anorm2 = p->anorm2;
    return DL_OK;
}

// ---------------------------------------------------------------------------
// argument blocks
// ---------------------------------------------------------------------------
namespace dlh {

GradArgs grad_args(const dl_problem* p, const double* lam, const double* gamma_ptr, double gamma_val,
                   const int32_t* done, double* X)
{
    GradArgs g;
    std::memset(&g, 0, sizeof g);
    g.A = p->A;
    g.C = p->C;
    g.dst = p->dst;
    g.U = p->U;
    g.IV = p->IV;
    g.perm = p->perm;
    g.X = X;
    g.items = p->items;
    g.chunks = p->chunks;
    g.lam = lam;
    g.gamma_ptr = gamma_ptr;
    g.gamma_val = gamma_val;
    g.done = done;
    g.J = p->J;
    g.K = p->K;
    g.Kc = p->Kc;
    g.nchunks = p->nchunks;
    g.part = p->part;
    g.tail = p->tail;
    g.obj_part = p->obj_part;
    g.det = p->det;
    for (int q = 0; q < 3; ++q) g.qs[q] = p->qs[q];
    g.nf = p->nf;
    for (int f = 0; f + 1 < kMfPlanes; ++f) {
        g.A2[f] = p->A2[f];
        g.dst2[f] = p->dst2[f];
    }
    g.restore = 0;
    g.dense_f = p->dense_f;
    g.dense_row = p->dense_row;
    g.srow = p->srow;
    g.corr_part = p->corr_part;
    return g;
}

ReduceArgs reduce_args(const dl_problem* p, int check, int mode, const double* lam,
                       const double* gamma_ptr, double gamma_val, const int32_t* done, double* grad_out)
{
    ReduceArgs r;
    std::memset(&r, 0, sizeof r);
    r.part = p->part;
    r.nchunks = p->nchunks;
    r.K = p->K;
    r.Kc = p->Kc;
    r.J = p->J;
    r.check = check;
    r.mode = mode;
    r.tail = p->tail;
    r.b = p->b;
    r.D = p->D;
    r.lam = lam;
    r.y = p->y;
    r.yp = p->yp;
    r.Gp = p->Gp;
    r.G = p->G;
    r.orig = p->orig;
    r.grad_out = grad_out;
    r.gamma_ptr = gamma_ptr;
    r.gamma_val = gamma_val;
    r.done = done;
    r.blockpart = p->blockpart;
    r.det = p->det;
    for (int q = 0; q < 3; ++q) r.iqs[q] = 1.0 / p->qs[q];
    r.srow = check && p->nf > 1 ? p->srow : nullptr;
    return r;
}

AgdArgs agd_args(const dl_problem* p, const SolveParams& prm, int check, double* trace)
{
    AgdArgs a;
    std::memset(&a, 0, sizeof a);
    a.st = p->st;
    a.prm = prm;
    a.check = check;
    a.nchunks = p->nchunks;
    a.nblk = p->nblk2;
    a.J = p->J;
    a.obj_part = p->obj_part;
    a.blockpart = p->blockpart;
    a.lam = p->lam;
    a.y = p->y;
    a.yp = p->yp;
    a.G = p->G;
    a.Gp = p->Gp;
    a.lam_eval = p->lam_eval;
    a.D = p->D;
    a.trace = trace;
    a.corr_part = p->nf > 1 ? p->corr_part : nullptr;
    return a;
}

hipError_t enqueue_iteration(dl_problem* p, const SolveParams& prm, int check, double* trace, hipStream_t s,
                             hipEvent_t ev0, hipEvent_t ev1)
{
    const double* gptr = &p->st->gamma;
    const int32_t* done = &p->st->done;
    GradArgs g = grad_args(p, p->lam_eval, gptr, 0.0, done, nullptr);
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
    if ((e = launch_grad(g, p->storage, check != 0, p->has_w != 0, p->has_cut != 0, s)) != hipSuccess) return e;
    if (ev1 && (e = hipEventRecord(ev1, s)) != hipSuccess) return e;
    ReduceArgs r = reduce_args(p, check, 0, p->lam_eval, gptr, 0.0, done, nullptr);
    AgdArgs a = agd_args(p, prm, check, trace);
    if ((e = launch_reduce(r, p->nblk2, s)) != hipSuccess) return e;
    if (check && p->nf > 1) {
        // the gap's restoration over each edge's rows (multi-entry columns)
        GradArgs gr = g;
        gr.restore = 1;
        if ((e = launch_grad(gr, p->storage, false, p->has_w != 0, p->has_cut != 0, s)) != hipSuccess) return e;
    }
    return launch_agd(a, s);
}

dl_status check_solve_opts(const dl_solve_opts* o)
{
    if (!o) { set_error("opts is NULL"); return DL_ERR_INVALID_ARG; }
    if (!(o->gamma0 > 0.0) || !(o->gamma_final > 0.0) || !std::isfinite(o->gamma0) || !std::isfinite(o->gamma_final)) {
        set_error("gamma0 and gamma_final must be positive"); return DL_ERR_INVALID_ARG;
    }
    if (o->n_stages < 1) { set_error("n_stages must be >= 1"); return DL_ERR_INVALID_ARG; }
    if (o->max_iters < 0 || o->check_every < 0 || o->stage_iters < 0) { set_error("negative iteration count"); return DL_ERR_INVALID_ARG; }
    if (!(o->max_step > 0.0) || !(o->init_step > 0.0)) { set_error("steps must be positive"); return DL_ERR_INVALID_ARG; }
    if (std::isnan(o->tol_rel_gap) || !(o->stage_tol >= 0.0)) { set_error("invalid tolerance"); return DL_ERR_INVALID_ARG; }
    if (o->graph_iters < 0) { set_error("graph_iters must be >= 0"); return DL_ERR_INVALID_ARG; }
    if (o->preset < DL_PRESET_CUSTOM || o->preset > DL_PRESET_NATURAL) { set_error("unknown preset %d", (int)o->preset); return DL_ERR_INVALID_ARG; }
    return DL_OK;
}

SolveParams make_params(const dl_solve_opts* o_in, const dl_problem* p)
{
    dl_solve_opts ob = *o_in;
    const dl_solve_opts* o = &ob;
    (void)dl_solve_opts_apply_preset(&ob, p->anorm2);   // options were checked before
    SolveParams P;
    std::memset(&P, 0, sizeof P);
    P.gamma0 = o->gamma0;
    P.gamma_final = o->n_stages > 1 ? o->gamma_final : o->gamma0;
    P.stage_tol = o->stage_tol;
    P.tol = o->tol_rel_gap;
    P.max_step = o->max_step;
    P.init_step = o->init_step;
    P.stage_iters = o->stage_iters;
    P.max_iters = o->max_iters;
    P.check_every = o->check_every;
    P.n_stages = o->n_stages;
    P.momentum = o->momentum;
    P.adaptive = o->adaptive;
    return P;
}

bool is_check_iter(const dl_solve_opts* o, int64_t k)
{
    return o->check_every > 0 && ((k + 1) % o->check_every == 0 || k + 1 == o->max_iters);
}

}  // namespace dlh

// ---------------------------------------------------------------------------
// dual evaluation
// ---------------------------------------------------------------------------
extern "C" dl_status dl_dual_grad(dl_problem* p, const double* lambda_dev, double gamma, double* grad_dev,
                                  double* x_dev, dl_eval* eval_host, void* hip_stream)
{
    if (!p || !lambda_dev || !grad_dev) { set_error("NULL argument"); return DL_ERR_INVALID_ARG; }
    if (!(gamma > 0.0) || !std::isfinite(gamma)) { set_error("gamma must be positive and finite"); return DL_ERR_INVALID_ARG; }
    hipStream_t s = (hipStream_t)hip_stream;
    const int check = eval_host ? 1 : 0;
    HIP_TRY(dl::launch_permute_in(lambda_dev, p->orig, p->J, p->lam_int, s), "permute lambda");
    GradArgs g = dlh::grad_args(p, p->lam_int, nullptr, gamma, nullptr, x_dev);
    HIP_TRY(launch_grad(g, p->storage, check != 0, p->has_w != 0, p->has_cut != 0, s), "gradient kernel");
    ReduceArgs r = dlh::reduce_args(p, check, 1, p->lam_int, nullptr, gamma, nullptr, grad_dev);
    HIP_TRY(launch_reduce(r, p->nblk2, s), "reduce kernel");
    if (eval_host) {
        if (p->nf > 1) {
            GradArgs gr = dlh::grad_args(p, p->lam_int, nullptr, gamma, nullptr, nullptr);
            gr.restore = 1;
            HIP_TRY(launch_grad(gr, p->storage, false, p->has_w != 0, p->has_cut != 0, s), "restoration pass");
        }
        HIP_TRY(launch_eval_finish(p->obj_part, p->nchunks, p->blockpart, p->nblk2, 1, gamma, p->eval6, s,
                                   p->nf > 1 ? p->corr_part : nullptr),
                "evaluation kernel");
        double h[8];
        HIP_TRY(hipMemcpyAsync(h, p->eval6, 6 * sizeof(double), hipMemcpyDeviceToHost, s), "copy scalars");
        HIP_TRY(hipStreamSynchronize(s), "synchronize");
        eval_host->g = h[0];
        eval_host->cx = h[1];
        eval_host->reg = h[2];
        eval_host->P = h[3];
        eval_host->rel_gap = h[4];
        eval_host->max_infeas = h[5];
    }
    return DL_OK;
}

extern "C" dl_status dl_time_grad_kernel(dl_problem* p, const double* lambda_dev, double gamma, int32_t iters,
                                         int32_t check, double* ms_per_launch, void* hip_stream)
{
    if (!p || !lambda_dev || !ms_per_launch || iters < 1) { set_error("invalid argument"); return DL_ERR_INVALID_ARG; }
    if (!(gamma > 0.0)) { set_error("gamma must be positive"); return DL_ERR_INVALID_ARG; }
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(dl::launch_permute_in(lambda_dev, p->orig, p->J, p->lam_int, s), "permute lambda");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "event");
    HIP_TRY(hipEventCreate(&e1), "event");
    float tot = 0.0f;
    dl_status st = DL_OK;
    for (int i = 0; i < iters && st == DL_OK; ++i) {
        GradArgs g = dlh::grad_args(p, p->lam_int, nullptr, gamma, nullptr, nullptr);
        hipError_t e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch_grad(g, p->storage, check != 0, p->has_w != 0, p->has_cut != 0, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        ReduceArgs r = dlh::reduce_args(p, check, 1, p->lam_int, nullptr, gamma, nullptr, p->lam);
        if (e == hipSuccess) e = launch_reduce(r, p->nblk2, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) st = hip_fail(e, "timing");
        tot += ms;
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == DL_OK) *ms_per_launch = tot / iters;
    return st;
}
