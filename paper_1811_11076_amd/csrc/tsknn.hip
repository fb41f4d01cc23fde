// tsknn: host runtime and C-ABI for the exact k-NN scan (arXiv 1811.11076)
// on gfx950.  All arithmetic of the method runs in the kernels of
// kernels.hpp; this file validates arguments, owns device memory and
// sequences launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "launch.hpp"
#include "model.hpp"
#include "runtime.hpp"
#include "tsknn.h"

using namespace tsk;

// ------------------------------------------------------------------ errors
namespace tsk {
thread_local std::string g_err;

int set_err(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
} // namespace tsk

struct Workspace {
    DevBuf<uint32_t> tau;
    DevBuf<unsigned long long> seedslots, ubslots, resslots;
    DevBuf<float> lbv;
    DevBuf<int32_t> surv, surv_cnt, max_cnt, qcur;
    DevBuf<int32_t> surv2;    // survivors re-ranked by LB_Box (DTW cascade)
    DevBuf<int32_t> segcnt;   // survivors per segment of SEG_LEN candidates [q][seg]
    DevBuf<int32_t> hist;     // survivors per bound bucket [q][SURV_BUCKETS]
    DevBuf<unsigned long long> segkey; // seed-set segment minima [q][SEEDSEG_MAX]
    DevBuf<float> rng;            // range query hit map [q][N]
    DevBuf<int64_t> rcnt, rqoff;  // its per-query counts and output offsets
    DevBuf<unsigned long long> ctr, work;
    DevBuf<int64_t> qoff;
    // the offsets of the chunk being enqueued (qoff + its first query): the
    // k-NN call uploads every query's offsets once
    int64_t *qoff_cur = nullptr;
    DevBuf<float> env;
    DevBuf<float> qdims;      // the queries padded to the kernels' dimension
    DevBuf<float> cenv;       // candidate envelopes [N][n][2][D] (option lb_both)
    DevBuf<float> tbuf;
    DevBuf<float> qpad;
    DevBuf<int2> fb;
    DevBuf<float> qtab;       // per-query sparse tables (length buckets)
    DevBuf<int64_t> qtab_off; // their offsets (floats)
    std::vector<int64_t> h_qoff, h_qtab;
    void release()
    {
        tau.release();
        seedslots.release();
        ubslots.release();
        resslots.release();
        lbv.release();
        surv.release();
        surv2.release();
        segcnt.release();
        hist.release();
        segkey.release();
        surv_cnt.release();
        max_cnt.release();
        qcur.release();
        rng.release();
        rcnt.release();
        rqoff.release();
        ctr.release();
        work.release();
        qoff.release();
        env.release();
        qdims.release();
        cenv.release();
        tbuf.release();
        qpad.release();
        fb.release();
        qtab.release();
        qtab_off.release();
    }
};

// Stage marks recorded per chunk when timing: start, after the learned
// order, after seed, after the bound kernel, after compaction (+ walks),
// after query staging, after the fast DP, after the general DP, after the
// output kernel.
constexpr int NEV = 9;

struct tsk_index {
    int device = 0;
    int64_t ws_limit = 0; // workspace bound of a query call (0 = none)
    int dim = 0;  // the kernels' dimension (kernel_dim of udim: padded above 8)
    int udim = 0; // the caller's dimension
    int64_t n = 0;
    int64_t total = 0;
    int32_t min_len = 0, max_len = 0;
    int n_cu = 256;
    std::vector<int64_t> h_off;
    std::vector<int32_t> h_len;
    float *aos = nullptr;
    int64_t *off = nullptr;
    int32_t *len = nullptr;
    int64_t n_tiles = 0;
    float *soa = nullptr;
    int64_t *tile_off = nullptr;
    int32_t *tile_len = nullptr;
    // length buckets (only when the series differ in length): ids sorted by
    // (length, id), tiles of <= 64 series of one length, SoA per tile
    bool bucketed = false;
    int32_t *perm = nullptr, *inv = nullptr;
    int32_t *bt_pos = nullptr, *bt_cnt = nullptr, *bt_len = nullptr;
    int64_t *bt_off = nullptr;
    float *bsoa = nullptr;
    int64_t n_btiles = 0;
    // candidate embeddings of the encoder (uid, version) last used for
    // TSK_ORDER_LEARNED
    DevBuf<float> emb;
    uint64_t emb_uid = 0, emb_version = 0;
    DevBuf<float> qemb;
    DevBuf<int32_t> lorder;
    // executable graph of the last use_graph call and what it was built for
    hipGraphExec_t graph_exec = nullptr;
    std::vector<int64_t> graph_key;
    int64_t graph_builds = 0;
    hipEvent_t gev[2] = {nullptr, nullptr};
    hipStream_t cap_stream = nullptr; // capture-only stream of use_graph
    // tsk_tune's choices per (dist, band mode, band r, band frac bits, k)
    std::map<std::array<int64_t, 5>, tsk_query_opts> tune_cache;
    hipStream_t last_stream = nullptr;
    Workspace ws;
    std::mutex mu;
    // profile accumulated by calls with opts->profile = 1
    std::vector<std::array<hipEvent_t, NEV>> ev_pool;
    size_t ev_used = 0;
    DevBuf<unsigned long long> prof_ctr;
    int64_t prof_calls = 0;
    int64_t prof_chunks = 0;
};

static int take_events(tsk_index *ix, hipEvent_t **out)
{
    if (ix->ev_used == ix->ev_pool.size()) {
        std::array<hipEvent_t, NEV> e;
        for (auto &x : e)
            HIP_TRY(hipEventCreate(&x));
        ix->ev_pool.push_back(e);
    }
    *out = ix->ev_pool[ix->ev_used++].data();
    return TSK_OK;
}

static void stats_from(tsk_stats *st, const unsigned long long *c)
{
    st->pairs = (int64_t)c[C_PAIRS];
    st->seed_pairs = (int64_t)c[C_SEED_PAIRS];
    st->bound_pruned = (int64_t)c[C_BOUND_PRUNED];
    st->dp_started = (int64_t)c[C_DP_STARTED];
    st->dp_completed = (int64_t)c[C_DP_COMPLETED];
    st->dp_abandoned = (int64_t)c[C_DP_ABANDONED];
    st->dp_cells = (int64_t)c[C_DP_CELLS];
    st->bound_steps = (int64_t)c[C_BOUND_STEPS];
    st->fallback_pairs = (int64_t)c[C_FALLBACK];
    st->dp_valid_cells = (int64_t)c[C_VALID_CELLS];
    st->dp_valid_cells_general = (int64_t)c[C_VALID_GEN];
    st->seed_steps = (int64_t)c[C_SEED_STEPS];
}

// Stage times of event sets [from, to) of the pool (synchronising):
// t[i] = sum of elapsed(mark i, mark i+1).
static int sum_events(tsk_index *ix, size_t from, size_t to, float t[NEV - 1])
{
    for (int i = 0; i < NEV - 1; ++i)
        t[i] = 0.0f;
    for (size_t i = from; i < to; ++i) {
        hipEvent_t *e = ix->ev_pool[i].data();
        HIP_TRY(hipEventSynchronize(e[NEV - 1]));
        for (int st = 0; st < NEV - 1; ++st) {
            float x = 0.0f;
            HIP_TRY(hipEventElapsedTime(&x, e[st], e[st + 1]));
            t[st] += x;
        }
    }
    return TSK_OK;
}

static void stats_times(tsk_stats *st, const float t[NEV - 1])
{
    st->ms_order = t[0];
    st->ms_seed = t[1];
    st->ms_bound_kernel = t[2];
    st->ms_bound = t[2] + t[3];
    st->ms_dp_fast = t[5];
    st->ms_dp_general = t[6];
    st->ms_dp = t[4] + t[5] + t[6];
    st->ms_final = t[7];
    st->ms_total = t[0] + t[1] + t[2] + t[3] + t[4] + t[5] + t[6] + t[7];
}

static uint32_t f_bits_host(float f)
{
    uint32_t u;
    memcpy(&u, &f, sizeof(u));
    return u;
}

// ------------------------------------------------------------------ dispatch
template <template <int> class F, typename... A> static void dispatch_d(int d, A &&...args)
{
    switch (d) {
    case 1: F<1>::run(args...); break;
    case 2: F<2>::run(args...); break;
    case 3: F<3>::run(args...); break;
    case 4: F<4>::run(args...); break;
    case 5: F<5>::run(args...); break;
    case 6: F<6>::run(args...); break;
    case 7: F<7>::run(args...); break;
    case 8: F<8>::run(args...); break;
    case 12: F<12>::run(args...); break;
    case 16: F<16>::run(args...); break;
    case 24: F<24>::run(args...); break;
    case 32: F<32>::run(args...); break;
    default: break;
    }
}

static int grid_for(int64_t n, int block, int cap = 1 << 16)
{
    int64_t g = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

static void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
}

static void fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
}

template <int D> struct PackLaunch {
    static void run(tsk_index *ix, const float *, hipStream_t s)
    {
        hipLaunchKernelGGL(k_pack_soa<D>, dim3((unsigned)ix->n_tiles), dim3(256), 0, s, ix->aos,
                           ix->off, ix->len, ix->n, ix->tile_off, ix->tile_len, ix->soa);
    }
};

// ------------------------------------------------------------------ validation helpers
static int check_series(const int64_t *off, int64_t n, const char *what, int32_t *min_len,
                        int32_t *max_len)
{
    if (!off)
        return set_err(TSK_ERR_INVALID_ARG, "%s offsets are NULL", what);
    if (n < 1)
        return set_err(TSK_ERR_INVALID_ARG, "%s count must be >= 1", what);
    if (n > INT32_MAX)
        return set_err(TSK_ERR_UNSUPPORTED, "%s count above 2^31-1", what);
    if (off[0] != 0)
        return set_err(TSK_ERR_INVALID_ARG, "%s offsets[0] must be 0", what);
    int32_t mn = INT32_MAX, mx = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t L = off[i + 1] - off[i];
        if (L < 1)
            return set_err(TSK_ERR_INVALID_ARG, "%s %lld has length %lld (must be >= 1)", what,
                           (long long)i, (long long)L);
        if (L > TSK_MAX_LEN)
            return set_err(TSK_ERR_UNSUPPORTED, "%s %lld has length %lld > %d", what, (long long)i,
                           (long long)L, TSK_MAX_LEN);
        mn = std::min<int32_t>(mn, (int32_t)L);
        mx = std::max<int32_t>(mx, (int32_t)L);
    }
    if (min_len)
        *min_len = mn;
    if (max_len)
        *max_len = mx;
    return TSK_OK;
}

static int check_band(tsk_band b)
{
    if (b.mode != TSK_BAND_NONE && b.mode != TSK_BAND_ABS && b.mode != TSK_BAND_FRAC)
        return set_err(TSK_ERR_INVALID_ARG, "band.mode %d is not NONE/ABS/FRAC", b.mode);
    if (b.mode == TSK_BAND_ABS && b.r < 0)
        return set_err(TSK_ERR_INVALID_ARG, "band.r must be >= 0");
    if (b.mode == TSK_BAND_FRAC && !(b.frac >= 0.0f && std::isfinite(b.frac)))
        return set_err(TSK_ERR_INVALID_ARG, "band.frac must be finite and >= 0");
    return TSK_OK;
}

static int check_device(const tsk_index *ix)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != ix->device)
        return set_err(TSK_ERR_INVALID_ARG, "current device %d differs from the index's device %d",
                       dev, ix->device);
    return TSK_OK;
}

// ------------------------------------------------------------------ C-ABI
extern "C" int tsk_version(int *major, int *minor)
{
    if (major)
        *major = TSK_VERSION_MAJOR;
    if (minor)
        *minor = TSK_VERSION_MINOR;
    return TSK_OK;
}

extern "C" const char *tsk_last_error(void) { return g_err.c_str(); }

extern "C" int tsk_index_info(const tsk_index *ix, int64_t *n_series, int32_t *dim)
{
    if (!ix)
        return set_err(TSK_ERR_INVALID_ARG, "index is NULL");
    if (n_series)
        *n_series = ix->n;
    if (dim)
        *dim = ix->udim;
    return TSK_OK;
}

static void free_index_memory(tsk_index *ix)
{
    if (ix->aos) (void)hipFree(ix->aos);
    if (ix->off) (void)hipFree(ix->off);
    if (ix->len) (void)hipFree(ix->len);
    if (ix->soa) (void)hipFree(ix->soa);
    if (ix->tile_off) (void)hipFree(ix->tile_off);
    if (ix->tile_len) (void)hipFree(ix->tile_len);
    for (int32_t *p : {ix->perm, ix->inv, ix->bt_pos, ix->bt_cnt, ix->bt_len})
        if (p) (void)hipFree(p);
    if (ix->bt_off) (void)hipFree(ix->bt_off);
    if (ix->bsoa) (void)hipFree(ix->bsoa);
    if (ix->graph_exec)
        (void)hipGraphExecDestroy(ix->graph_exec);
    for (auto &e : ix->gev)
        if (e)
            (void)hipEventDestroy(e);
    if (ix->cap_stream)
        (void)hipStreamDestroy(ix->cap_stream);
    ix->ws.release();
    ix->emb.release();
    ix->qemb.release();
    ix->lorder.release();
    ix->prof_ctr.release();
    for (auto &e : ix->ev_pool)
        for (auto &x : e)
            (void)hipEventDestroy(x);
    ix->ev_pool.clear();
}

// first non-finite element: grid-stride, atomic minimum of the index
static __global__ void k_first_nonfinite(const float *__restrict__ v, int64_t n,
                                         unsigned long long *first)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!__builtin_isfinite(v[i]))
            atomicMin(first, (unsigned long long)i);
}

extern "C" int tsk_validate_values(const float *values_dev, int64_t count, int64_t *first_bad_host,
                                   void *hip_stream)
{
    g_err.clear();
    if (first_bad_host)
        *first_bad_host = -1;
    if (count < 0)
        return set_err(TSK_ERR_INVALID_ARG, "count must be >= 0");
    if (count == 0)
        return TSK_OK;
    if (!values_dev)
        return set_err(TSK_ERR_INVALID_ARG, "values_dev is NULL");
    TSK_TRY(check_dev_ptr(values_dev, -1, "values_dev"));
    hipStream_t s = (hipStream_t)hip_stream;
    DevBuf<unsigned long long> first;
    TSK_TRY(first.ensure(1));
    fill_u64(first.p, ~0ull, 1, s);
    hipLaunchKernelGGL(k_first_nonfinite, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s,
                       values_dev, count, first.p);
    unsigned long long h = ~0ull;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(&h, first.p, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    first.release();
    if (e != hipSuccess)
        return set_err(TSK_ERR_DEVICE, "validate: %s", hipGetErrorString(e));
    if (h == ~0ull)
        return TSK_OK;
    if (first_bad_host)
        *first_bad_host = (int64_t)h;
    return set_err(TSK_ERR_INVALID_ARG, "value %lld is not finite", (long long)h);
}

extern "C" int tsk_index_free(tsk_index *ix)
{
    if (!ix)
        return TSK_OK;
    (void)hipDeviceSynchronize();
    free_index_memory(ix);
    delete ix;
    return TSK_OK;
}

static BucketArgs bucket_args(const tsk_index *ix)
{
    BucketArgs b;
    b.perm = ix->perm;
    b.tpos = ix->bt_pos;
    b.tcnt = ix->bt_cnt;
    b.tlen = ix->bt_len;
    b.toff = ix->bt_off;
    b.soa = ix->bsoa;
    b.n_tiles = ix->n_btiles;
    return b;
}

static int index_build_impl(tsk_index *ix, const float *values_dev, hipStream_t s)
{
    const int D = ix->dim;
    HIP_TRY(hipMalloc((void **)&ix->aos, std::max<int64_t>(1, ix->total * D) * sizeof(float)));
    HIP_TRY(hipMalloc((void **)&ix->off, (ix->n + 1) * sizeof(int64_t)));
    HIP_TRY(hipMalloc((void **)&ix->len, ix->n * sizeof(int32_t)));
    if (ix->udim == D) {
        HIP_TRY(hipMemcpyAsync(ix->aos, values_dev, ix->total * D * sizeof(float),
                               hipMemcpyDeviceToDevice, s));
    } else {
        hipLaunchKernelGGL(k_pad_dims, dim3(grid_for(ix->total * D, 256, 8192)), dim3(256), 0, s,
                           values_dev, ix->total, ix->udim, D, ix->aos);
    }
    HIP_TRY(hipMemcpyAsync(ix->off, ix->h_off.data(), (ix->n + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ix->len, ix->h_len.data(), ix->n * sizeof(int32_t),
                           hipMemcpyHostToDevice, s));
    ix->n_tiles = (ix->n + 63) / 64;
    std::vector<int64_t> toff(ix->n_tiles + 1, 0);
    std::vector<int32_t> tlen(ix->n_tiles, 0);
    for (int64_t t = 0; t < ix->n_tiles; ++t) {
        int32_t mx = 0;
        for (int64_t c = t * 64; c < std::min<int64_t>(ix->n, t * 64 + 64); ++c)
            mx = std::max(mx, ix->h_len[c]);
        tlen[t] = mx;
        toff[t + 1] = toff[t] + (int64_t)mx * D * 64;
    }
    HIP_TRY(hipMalloc((void **)&ix->soa, std::max<int64_t>(1, toff.back()) * sizeof(float)));
    HIP_TRY(hipMalloc((void **)&ix->tile_off, toff.size() * sizeof(int64_t)));
    HIP_TRY(hipMalloc((void **)&ix->tile_len, tlen.size() * sizeof(int32_t)));
    HIP_TRY(hipMemcpyAsync(ix->tile_off, toff.data(), toff.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ix->tile_len, tlen.data(), tlen.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s));
    dispatch_d<PackLaunch>(D, ix, values_dev, s);
    HIP_TRY(hipGetLastError());
    std::vector<int32_t> perm, inv, bpos, bcnt, blen;
    std::vector<int64_t> boff;
    if (ix->min_len != ix->max_len) {
        // length buckets for the bound pass of uneven-length DTW
        perm.resize(ix->n);
        for (int64_t i = 0; i < ix->n; ++i)
            perm[i] = (int32_t)i;
        std::stable_sort(perm.begin(), perm.end(),
                         [&](int32_t a, int32_t b) { return ix->h_len[a] < ix->h_len[b]; });
        inv.resize(ix->n);
        for (int64_t p = 0; p < ix->n; ++p)
            inv[perm[p]] = (int32_t)p;
        boff.push_back(0);
        for (int64_t p = 0; p < ix->n;) {
            const int32_t L = ix->h_len[perm[p]];
            int64_t e = p;
            while (e < ix->n && e - p < 64 && ix->h_len[perm[e]] == L)
                ++e;
            bpos.push_back((int32_t)p);
            bcnt.push_back((int32_t)(e - p));
            blen.push_back(L);
            boff.push_back(boff.back() + (int64_t)L * D * 64);
            p = e;
        }
        ix->n_btiles = (int64_t)bpos.size();
        const size_t nt = (size_t)ix->n_btiles;
        HIP_TRY(hipMalloc((void **)&ix->perm, ix->n * sizeof(int32_t)));
        HIP_TRY(hipMalloc((void **)&ix->inv, ix->n * sizeof(int32_t)));
        HIP_TRY(hipMalloc((void **)&ix->bt_pos, nt * sizeof(int32_t)));
        HIP_TRY(hipMalloc((void **)&ix->bt_cnt, nt * sizeof(int32_t)));
        HIP_TRY(hipMalloc((void **)&ix->bt_len, nt * sizeof(int32_t)));
        HIP_TRY(hipMalloc((void **)&ix->bt_off, (nt + 1) * sizeof(int64_t)));
        HIP_TRY(hipMalloc((void **)&ix->bsoa, boff.back() * sizeof(float)));
        HIP_TRY(hipMemcpyAsync(ix->perm, perm.data(), ix->n * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ix->inv, inv.data(), ix->n * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ix->bt_pos, bpos.data(), nt * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ix->bt_cnt, bcnt.data(), nt * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ix->bt_len, blen.data(), nt * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ix->bt_off, boff.data(), (nt + 1) * sizeof(int64_t),
                               hipMemcpyHostToDevice, s));
        ix->bucketed = true;
        launch_pack_bucket(D, ix->aos, ix->off, bucket_args(ix), ix->bsoa, s);
        HIP_TRY(hipGetLastError());
    }
    // the host vectors feeding the async copies live in the index; wait so
    // the caller may release its input as soon as this call returns
    HIP_TRY(hipStreamSynchronize(s));
    return TSK_OK;
}

extern "C" int tsk_index_build(const float *values_dev, const int64_t *offsets_host,
                               int64_t n_series, int32_t dim, const tsk_index_opts *opts,
                               void *hip_stream, tsk_index **out)
{
    g_err.clear();
    if (!out)
        return set_err(TSK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!values_dev)
        return set_err(TSK_ERR_INVALID_ARG, "values_dev is NULL");
    if (dim < 1 || dim > TSK_MAX_DIM)
        return set_err(TSK_ERR_UNSUPPORTED, "dim %d outside [1, %d]", dim, TSK_MAX_DIM);
    if (opts && opts->size != (int64_t)sizeof(tsk_index_opts))
        return set_err(TSK_ERR_INVALID_ARG, "opts->size mismatch");
    if (opts && opts->workspace_limit_bytes < 0)
        return set_err(TSK_ERR_INVALID_ARG, "workspace_limit_bytes must be >= 0");
    int32_t mn = 0, mx = 0;
    TSK_TRY(check_series(offsets_host, n_series, "series", &mn, &mx));
    int dev = 0, ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return set_err(TSK_ERR_DEVICE, "no HIP device available");
    }
    HIP_TRY(hipGetDevice(&dev));
    TSK_TRY(check_dev_ptr(values_dev, dev, "values_dev"));
    tsk_index *ix = new (std::nothrow) tsk_index();
    if (!ix)
        return set_err(TSK_ERR_OOM, "host allocation failed");
    ix->device = dev;
    ix->ws_limit = opts ? opts->workspace_limit_bytes : 0;
    ix->udim = dim;
    ix->dim = kernel_dim(dim);
    ix->n = n_series;
    ix->total = offsets_host[n_series];
    ix->min_len = mn;
    ix->max_len = mx;
    ix->h_off.assign(offsets_host, offsets_host + n_series + 1);
    ix->h_len.resize(n_series);
    for (int64_t i = 0; i < n_series; ++i)
        ix->h_len[i] = (int32_t)(offsets_host[i + 1] - offsets_host[i]);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess)
        ix->n_cu = std::max(1, prop.multiProcessorCount);
    int rc = index_build_impl(ix, values_dev, (hipStream_t)hip_stream);
    if (rc != TSK_OK) {
        free_index_memory(ix);
        delete ix;
        return rc;
    }
    *out = ix;
    return TSK_OK;
}

// ------------------------------------------------------------------ query plumbing
struct QueryPlan {
    int D;
    int dist;
    int k;
    BandArgs ba;
    int64_t nq, N;
    int64_t chunk;
    int seed;
    const int32_t *order;
    bool env_ok;
};

template <int D> struct EnvLaunch {
    static void run(tsk_index *ix, const float *qv, int nq, BandArgs ba, hipStream_t s)
    {
        const int n = ix->max_len;
        hipLaunchKernelGGL(k_env<D>, dim3((n + 63) / 64, nq), dim3(64), 0, s, qv, ix->ws.qoff_cur, nq,
                           n, ba, ix->ws.env.p);
    }
};

template <int D> struct SeedLaunch {
    static void run(tsk_index *ix, const float *qv, int nq, const QueryPlan &P,
                    const int32_t *order, hipStream_t s)
    {
        if (P.seed <= 0)
            return;
        dim3 grid((P.seed + 63) / 64, nq);
        if (P.dist == DIST_DK)
            hipLaunchKernelGGL((k_seed<D, DIST_DK>), grid, dim3(64), 0, s, qv, ix->ws.qoff_cur, nq,
                               ix->aos, ix->off, ix->len, ix->n, order, P.seed, P.k, P.ba,
                               ix->ws.seedslots.p, ix->ws.tau.p, ix->ws.ctr.p);
        else
            hipLaunchKernelGGL((k_seed<D, DIST_DTW>), grid, dim3(64), 0, s, qv, ix->ws.qoff_cur, nq,
                               ix->aos, ix->off, ix->len, ix->n, order, P.seed, P.k, P.ba,
                               ix->ws.seedslots.p, ix->ws.tau.p, ix->ws.ctr.p);
    }
};

static BoundArgs bound_args(tsk_index *ix, const float *qv, int nq, const QueryPlan &P)
{
    BoundArgs a;
    a.qv = qv;
    a.qoff = ix->ws.qoff_cur;
    a.nq = nq;
    a.qgroup = 4;
    a.soa = ix->soa;
    a.tile_off = ix->tile_off;
    a.aos = ix->aos;
    a.off = ix->off;
    a.len = ix->len;
    a.N = ix->n;
    a.k = P.k;
    a.ba = P.ba;
    a.env = P.env_ok ? ix->ws.env.p : nullptr;
    a.env_n = ix->max_len;
    a.lb_prefix = 0;
    a.tau = ix->ws.tau.p;
    a.ubslots = ix->ws.ubslots.p;
    a.lbv = ix->ws.lbv.p;
    a.ctr = ix->ws.ctr.p;
    a.dbg_lb = nullptr;
    a.dbg_ub = nullptr;
    a.dbg_steps = nullptr;
    return a;
}

template <int D> struct BoundLaunch {
    static void run(const BoundArgs &a, int dist, bool debug, hipStream_t s)
    {
        dim3 grid((unsigned)((a.N + 255) / 256), (unsigned)((a.nq + a.qgroup - 1) / a.qgroup));
        if (dist == DIST_DK) {
            if (debug)
                hipLaunchKernelGGL((k_bounds<D, DIST_DK, true>), grid, dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((k_bounds<D, DIST_DK, false>), grid, dim3(256), 0, s, a);
        } else {
            if (debug)
                hipLaunchKernelGGL((k_bounds<D, DIST_DTW, true>), grid, dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((k_bounds<D, DIST_DTW, false>), grid, dim3(256), 0, s, a);
        }
    }
};

static DpArgs dp_args(tsk_index *ix, const float *qv, int nq, const QueryPlan &P)
{
    DpArgs a;
    a.qv = qv;
    a.qoff = ix->ws.qoff_cur;
    a.nq = nq;
    a.aos = ix->aos;
    a.off = ix->off;
    a.len = ix->len;
    a.N = ix->n;
    a.k = P.k;
    a.ba = P.ba;
    a.tau = ix->ws.tau.p;
    a.lbv = ix->ws.lbv.p;
    a.lb_inv = nullptr;
    a.surv = ix->ws.surv.p;
    a.surv_cnt = ix->ws.surv_cnt.p;
    a.max_cnt = ix->ws.max_cnt.p;
    a.resslots = ix->ws.resslots.p;
    a.work = ix->ws.work.p;
    a.tbuf = ix->ws.tbuf.p;
    a.tb_stride = 2 * ix->max_len;
    a.ctr = ix->ws.ctr.p;
    a.out_all = nullptr;
    a.fb = ix->ws.fb.p;
    a.fb_count = ix->ws.work.p + 1;
    // one row per lane wastes fewer out-of-band cells on narrow bands but
    // costs more per cell; four measured faster on the class-warp bands
    a.rows_per_lane = 4;
    a.range_out = nullptr;
    return a;
}

static int dp_blocks(const tsk_index *ix) { return ix->n_cu * 4; }

// Which lane-per-pair kernel serves a call (0 = none: everything goes to the
// general DP).
enum { FAST_NONE = 0, FAST_BAND, FAST_TUBE32, FAST_BAND_DKV };

static FastArgs fast_args(tsk_index *ix, int nq, const QueryPlan &P, int qrows)
{
    FastArgs a;
    a.qoff = ix->ws.qoff_cur;
    a.nq = nq;
    a.aos = ix->aos;
    a.off = ix->off;
    a.len = ix->len;
    a.N = ix->n;
    a.k = P.k;
    a.ba = P.ba;
    a.tau = ix->ws.tau.p;
    a.lbv = ix->ws.lbv.p;
    a.lb_inv = nullptr;
    a.surv = ix->ws.surv.p;
    a.surv_cnt = ix->ws.surv_cnt.p;
    a.max_cnt = ix->ws.max_cnt.p;
    a.resslots = ix->ws.resslots.p;
    a.work = ix->ws.work.p;
    a.fb = ix->ws.fb.p;
    a.qpad = ix->ws.qpad.p;
    a.qrows = qrows;
    a.task = 64;
    a.qcur = ix->ws.qcur.p;
    a.range_out = nullptr;
    a.dk_virtual = 0;
    // query-interleaved: each query's survivors spread over the kernel's
    // lifetime, so later ones meet a tighter threshold (query-major
    // measured 1.6x slower on the banded DP)
    a.qmajor = 0;
    a.ctr = ix->ws.ctr.p;
    return a;
}

template <int D> struct QpadLaunch {
    static void run(const float *qv, const int64_t *qoff, int nq, int qrows, float *qpad,
                    hipStream_t s)
    {
        hipLaunchKernelGGL(k_qpad<D>, dim3((qrows + 63) / 64, nq), dim3(64), 0, s, qv, qoff, nq,
                           qrows, qpad);
    }
};

// Picks the lane-per-pair kernel from the call's shape (per-pair exceptions
// are handed to the general DP inside the kernels).
static int pick_fast(const tsk_index *ix, int dist, const tsk_band &band, int32_t qmin, int32_t qmax,
                     int dp_kernel, int dk_band_slots, int *wsel)
{
    *wsel = -1;
    // the lane-per-pair kernels are built for up to 8 dimensions
    if (dp_kernel == 1 || ix->dim > 8)
        return FAST_NONE;
    const int DP = pad_dim(ix->dim);
    if (dist == TSK_DK && band.mode == TSK_BAND_NONE && dk_band_slots > 0 && qmin == qmax &&
        ix->min_len == ix->max_len && ix->min_len == qmin) {
        for (int i = 0; i < N_BAND_WS; ++i)
            if (BAND_WS[i] == dk_band_slots) {
                *wsel = i;
                return FAST_BAND_DKV;
            }
    }
    if (dist == TSK_DK && band.mode == TSK_BAND_NONE) {
        if ((size_t)(qmax + 32) * DP * sizeof(float) <= 64 * 1024)
            return FAST_TUBE32;
        return FAST_NONE;
    }
    // banded (or unbanded short) equal-length pairs
    if (qmin != qmax || ix->min_len != ix->max_len || ix->min_len != qmin)
        return FAST_NONE;
    const int m = qmin;
    int w;
    if (band.mode == TSK_BAND_ABS)
        w = band.r;
    else if (band.mode == TSK_BAND_FRAC)
        w = (int)std::floor((double)band.frac * (double)m);
    else
        w = m - 1;
    w = std::min(w, m - 1);
    for (int i = 0; i < N_BAND_WS; ++i)
        if (2 * w + 1 <= BAND_WS[i]) {
            *wsel = (BAND_WS[i] == 52 && 2 * w + 1 >= 49) ? BAND_W52_TIGHT : i;
            return FAST_BAND;
        }
    return FAST_NONE;
}

static int check_queries(const tsk_index *ix, const float *qv, const int64_t *qoff, int64_t nq,
                         int32_t dist, tsk_band band)
{
    if (!ix)
        return set_err(TSK_ERR_INVALID_ARG, "index is NULL");
    if (!qv)
        return set_err(TSK_ERR_INVALID_ARG, "q_values_dev is NULL");
    TSK_TRY(check_series(qoff, nq, "query", nullptr, nullptr));
    if (dist != TSK_DTW && dist != TSK_DK)
        return set_err(TSK_ERR_INVALID_ARG, "dist %d is not TSK_DTW/TSK_DK", dist);
    TSK_TRY(check_band(band));
    TSK_TRY(check_device(ix));
    TSK_TRY(check_dev_ptr(qv, ix->device, "q_values_dev"));
    return TSK_OK;
}

// The queries as the kernels read them: the caller's values, or above 8
// dimensions a copy padded with zero coordinates (in the workspace).
static int kernel_queries(tsk_index *ix, const float *qv, const int64_t *qoff_host, int64_t nq,
                          hipStream_t s, const float **out)
{
    *out = qv;
    if (ix->udim == ix->dim)
        return TSK_OK;
    const int64_t rows = qoff_host[nq];
    TSK_TRY(ix->ws.qdims.ensure((size_t)rows * ix->dim));
    hipLaunchKernelGGL(k_pad_dims, dim3(grid_for(rows * ix->dim, 256, 8192)), dim3(256), 0, s, qv,
                       rows, ix->udim, ix->dim, ix->ws.qdims.p);
    HIP_TRY(hipGetLastError());
    *out = ix->ws.qdims.p;
    return TSK_OK;
}

// Workspace for a chunk of nq queries; sizes follow the index.
static int ensure_ws(tsk_index *ix, int64_t nq, int k, bool need_env, bool need_cenv = false,
                     bool need_surv2 = false)
{
    Workspace &w = ix->ws;
    const int64_t N = ix->n;
    TSK_TRY(w.tau.ensure(nq));
    TSK_TRY(w.seedslots.ensure(nq * k));
    TSK_TRY(w.ubslots.ensure(nq * k));
    TSK_TRY(w.resslots.ensure(nq * k));
    TSK_TRY(w.lbv.ensure(nq * N));
    TSK_TRY(w.surv.ensure(nq * N));
    if (need_surv2)
        TSK_TRY(w.surv2.ensure(nq * N));
    TSK_TRY(w.segcnt.ensure(nq * ((N + SEG_LEN - 1) / SEG_LEN)));
    TSK_TRY(w.hist.ensure(nq * SURV_BUCKETS));
    TSK_TRY(w.segkey.ensure(nq * SEEDSEG_MAX));
    TSK_TRY(w.surv_cnt.ensure(nq));
    TSK_TRY(w.max_cnt.ensure(1));
    TSK_TRY(w.qcur.ensure(nq));
    TSK_TRY(w.rcnt.ensure(nq));
    TSK_TRY(w.ctr.ensure(CTR_WORDS));
    TSK_TRY(w.work.ensure(8));
    TSK_TRY(w.qoff.ensure(nq + 1));
    if (need_env)
        TSK_TRY(w.env.ensure(nq * (int64_t)ix->max_len * 2 * ix->dim));
    if (need_cenv)
        TSK_TRY(w.cenv.ensure((size_t)N * ix->max_len * 2 * ix->dim));
    TSK_TRY(w.tbuf.ensure((size_t)dp_blocks(ix) * 4 * 2 * ix->max_len));
    TSK_TRY(w.fb.ensure(nq * N));
    return TSK_OK;
}

// Relative query offsets of queries [q0, q0+nq) to the device.
static int upload_qoff(tsk_index *ix, const int64_t *qoff, int64_t q0, int64_t nq, hipStream_t s)
{
    ix->ws.h_qoff.assign(qoff + q0, qoff + q0 + nq + 1);
    HIP_TRY(hipMemcpyAsync(ix->ws.qoff.p, ix->ws.h_qoff.data(), (nq + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    ix->ws.qoff_cur = ix->ws.qoff.p;
    return TSK_OK;
}

// Sparse-table offsets of a chunk's queries (length-bucket bound pass):
// host arithmetic, allocation and upload; the tables themselves are built
// by a kernel in the query sequence.
static int prepare_qtables(tsk_index *ix, const int64_t *qoff_host, int64_t q0, int nq,
                           hipStream_t s)
{
    const int DP = pad_dim(ix->dim);
    std::vector<int64_t> &h = ix->ws.h_qtab;
    h.assign(nq + 1, 0);
    for (int i = 0; i < nq; ++i)
        h[i + 1] = h[i] + qtable_floats((int)(qoff_host[q0 + i + 1] - qoff_host[q0 + i]), DP);
    TSK_TRY(ix->ws.qtab.ensure(h[nq]));
    TSK_TRY(ix->ws.qtab_off.ensure(nq + 1));
    HIP_TRY(hipMemcpyAsync(ix->ws.qtab_off.p, h.data(), (nq + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    return TSK_OK;
}

static int64_t chunk_queries(const tsk_index *ix, int64_t nq)
{
    // (query, candidate) entries per chunk: 2^30 (a workspace of about 24
    // bytes per entry, 26 GB at 10^6 series, which HBM holds); fewer, larger
    // chunks give the latency-bound seed walks and the DP launches more
    // work each (4096 x 10^6 x 512 x 6: 4 chunks of 1073 queries, DK 77 -> 64
    // and DTW 328 -> 318 ms per call against 16 chunks of 268)
    const int64_t budget = (int64_t)1 << 30;
    // at most 65535 queries: several kernels put the chunk's queries on the
    // grid's y dimension
    int64_t q = std::min<int64_t>(budget / std::max<int64_t>(1, ix->n), 65535);
    if (ix->ws_limit > 0) {
        // per query: bounds, survivors (two lists on equal lengths),
        // fallback pairs and range hits per series (24 bytes), the envelope
        // and staged rows per point
        const int64_t per_q = ix->n * 24 + (int64_t)ix->max_len * (8 * ix->dim + 32) + 1024;
        q = std::min<int64_t>(q, ix->ws_limit / per_q);
    }
    return std::max<int64_t>(1, std::min<int64_t>(nq, q));
}

static std::array<int64_t, 5> tune_key(int32_t dist, tsk_band band, int32_t k)
{
    return {dist, band.mode, band.r, (int64_t)f_bits_host(band.frac), k};
}

// The fields tsk_tune chooses.
static void apply_tuned(tsk_query_opts *o, const tsk_query_opts &t)
{
    o->seed_count = t.seed_count;
    o->tube_rows = t.tube_rows;
    o->task_size = t.task_size;
    o->walk_pass = t.walk_pass;
    o->lb_qgroup = t.lb_qgroup;
    o->dk_band_slots = t.dk_band_slots;
    o->surv_order = t.surv_order;
    o->dp_rows = t.dp_rows;
    o->dp_waves_per_cu = t.dp_waves_per_cu;
    o->dk_seed = t.dk_seed;
    o->bound_seed = t.bound_seed;
    o->dtw_cascade = t.dtw_cascade;
    o->dk_box = t.dk_box;
    o->lb_prefix = t.lb_prefix;
}

// A range query (fixed threshold, every hit reported) riding on the k-NN
// pipeline: the threshold never tightens, results go to a per-pair hit map.
struct RangeReq {
    float tau_key;    // largest key whose distance is within the radius
    int64_t capacity; // entries of ids / dist
    int64_t *ids;
    float *dist;
    int64_t *offsets_host; // [n_queries + 1]
};

// The workspace of one chunk of nq queries laid out in one region of
// memory, each buffer 256-byte aligned (the same buffers and sizes that
// ensure_ws and a chunk's preparation request).  With base == nullptr only
// the size is computed; otherwise the workspace's buffers borrow the region.
struct WsShape {
    int64_t nq;
    int64_t nq_total;        // queries of the call (their offsets are uploaded at once)
    int k;
    bool env, qpad, qtab, surv2;
    int qrows;               // staged rows per query (longest query + padding)
    int64_t qtab_floats_q;   // sparse-table floats of the longest query
    int64_t qdims_floats;    // the call's queries padded to the kernels' dimension
};
static size_t carve_ws(const tsk_index *ix, const WsShape &sh, char *base, Workspace *w)
{
    size_t off = 0;
    auto take = [&](auto &buf, size_t n) {
        using T = std::remove_pointer_t<decltype(buf.p)>;
        off = (off + 255) & ~(size_t)255;
        if (base)
            buf.borrow(reinterpret_cast<T *>(base + off), n);
        off += std::max<size_t>(n, 1) * sizeof(T);
    };
    const int64_t N = ix->n, nq = sh.nq;
    take(w->tau, nq);
    take(w->seedslots, nq * sh.k);
    take(w->ubslots, nq * sh.k);
    take(w->resslots, nq * sh.k);
    take(w->lbv, nq * N);
    take(w->surv, nq * N);
    if (sh.surv2)
        take(w->surv2, nq * N);
    take(w->segcnt, nq * ((N + SEG_LEN - 1) / SEG_LEN));
    take(w->hist, nq * SURV_BUCKETS);
    take(w->segkey, nq * SEEDSEG_MAX);
    take(w->surv_cnt, nq);
    take(w->max_cnt, 1);
    take(w->qcur, nq);
    take(w->rcnt, nq);
    take(w->ctr, CTR_WORDS);
    take(w->work, 8);
    take(w->qoff, sh.nq_total + 1);
    if (sh.env)
        take(w->env, nq * (int64_t)ix->max_len * 2 * ix->dim);
    take(w->tbuf, (size_t)dp_blocks(ix) * 4 * 2 * ix->max_len);
    take(w->fb, nq * N);
    if (sh.qpad)
        take(w->qpad, (size_t)nq * sh.qrows * pad_dim(ix->dim));
    if (sh.qdims_floats > 0)
        take(w->qdims, sh.qdims_floats);
    if (sh.qtab) {
        take(w->qtab, nq * sh.qtab_floats_q);
        take(w->qtab_off, nq + 1);
    }
    return off;
}

// Fixed device workspace of tsk_knn_query_noalloc.  Host code never uses
// the array's name as an address (it is a host-side stand-in there): the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[TSK_NOALLOC_SCRATCH_BYTES];
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// The calling thread's current device's copy of the array (the device is
// the index's: callers check that first).
static int scratch_address(int device, char **out)
{
    if (device < 0 || device >= SCRATCH_MAX_DEVICES)
        return set_err(TSK_ERR_UNSUPPORTED, "device %d outside the fixed workspace's table",
                       device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr)
            return set_err(TSK_ERR_DEVICE, "hipGetSymbolAddress gave a null fixed workspace");
        g_scratch_ptr[device] = (char *)ptr;
    }
    *out = g_scratch_ptr[device];
    return TSK_OK;
}

// A call whose workspace is carved from a fixed region instead of the
// index's growable buffers (nothing allocated on the device).
struct FixedWs {
    char *base;
    size_t bytes;
};

static int scan_impl(const tsk_index *cix, const float *q_values_dev,
                     const int64_t *q_offsets_host, int64_t n_queries, int32_t k, int32_t dist,
                     tsk_band band, const tsk_query_opts *opts, int64_t *out_ids_dev,
                     float *out_dist_dev, tsk_stats *stats_host, void *hip_stream,
                     const RangeReq *rr, const FixedWs *fx = nullptr)
{
    g_err.clear();
    TSK_TRY(check_queries(cix, q_values_dev, q_offsets_host, n_queries, dist, band));
    if (k < 1)
        return set_err(TSK_ERR_INVALID_ARG, "k must be >= 1");
    if (k > TSK_MAX_K)
        return set_err(TSK_ERR_UNSUPPORTED, "k %d > %d", k, TSK_MAX_K);
    if (!rr && (!out_ids_dev || !out_dist_dev))
        return set_err(TSK_ERR_INVALID_ARG, "output pointers are NULL");
    TSK_TRY(check_dev_ptr(out_ids_dev, cix->device, "out_ids_dev"));
    TSK_TRY(check_dev_ptr(out_dist_dev, cix->device, "out_dist_dev"));
    if (rr && rr->capacity > 0) {
        TSK_TRY(check_dev_ptr(rr->ids, cix->device, "out_ids_dev"));
        TSK_TRY(check_dev_ptr(rr->dist, cix->device, "out_dist_dev"));
    }
    tsk_query_opts o;
    memset(&o, 0, sizeof(o));
    o.walk_pass = -1;
    if (opts) {
        if (opts->size != (int64_t)sizeof(tsk_query_opts))
            return set_err(TSK_ERR_INVALID_ARG, "opts->size mismatch");
        o = *opts;
    }
    if (o.order != TSK_ORDER_PLAIN && o.order != TSK_ORDER_GIVEN && o.order != TSK_ORDER_LEARNED)
        return set_err(TSK_ERR_INVALID_ARG, "opts->order %d unknown", o.order);
    if (o.order == TSK_ORDER_GIVEN && !o.order_dev)
        return set_err(TSK_ERR_INVALID_ARG, "TSK_ORDER_GIVEN needs order_dev");
    if (o.order == TSK_ORDER_GIVEN)
        TSK_TRY(check_dev_ptr(o.order_dev, cix->device, "opts->order_dev"));
    if (o.order == TSK_ORDER_LEARNED) {
        if (!o.model)
            return set_err(TSK_ERR_INVALID_ARG, "TSK_ORDER_LEARNED needs opts->model");
        if (o.model->dim != cix->udim || o.model->device != cix->device)
            return set_err(TSK_ERR_INVALID_ARG, "the model's dim/device differ from the index's");
    }
    if (o.seed_count < 0)
        return set_err(TSK_ERR_INVALID_ARG, "seed_count must be >= 0");
    if (o.walk_pass < -1 || o.walk_pass > 1)
        return set_err(TSK_ERR_INVALID_ARG, "walk_pass must be -1, 0 or 1");
    if (o.task_size < 0 || o.task_size > (1 << 20))
        return set_err(TSK_ERR_INVALID_ARG, "task_size out of range");
    if (o.tube_rows != 0 && o.tube_rows != 8 && o.tube_rows != 16 && o.tube_rows != 32)
        return set_err(TSK_ERR_INVALID_ARG, "tube_rows must be 0, 8, 16 or 32");
    if (o.dk_band_slots != 0 && o.dk_band_slots != 32 && o.dk_band_slots != 56 &&
        o.dk_band_slots != 64 && o.dk_band_slots != 104 && o.dk_band_slots != 128)
        return set_err(TSK_ERR_INVALID_ARG, "dk_band_slots must be 0, 32, 56, 64, 104 or 128");
    if (o.dp_waves_per_cu != 0 && o.dp_waves_per_cu != 8 && o.dp_waves_per_cu != 16 &&
        o.dp_waves_per_cu != 32)
        return set_err(TSK_ERR_INVALID_ARG, "dp_waves_per_cu must be 0, 8, 16 or 32");
    if (o.dk_seed != 0 && o.dk_seed != 1)
        return set_err(TSK_ERR_INVALID_ARG, "dk_seed must be 0 or 1");
    if (o.dp_rows != 0 && o.dp_rows != 1 && o.dp_rows != 2 && o.dp_rows != 4)
        return set_err(TSK_ERR_INVALID_ARG, "dp_rows must be 0, 1, 2 or 4");
    if (o.surv_order < 0 || o.surv_order > 2)
        return set_err(TSK_ERR_INVALID_ARG, "surv_order must be 0, 1 or 2");
    if (o.lb_qgroup != 0 && o.lb_qgroup != 1 && o.lb_qgroup != 2 && o.lb_qgroup != 4 &&
        o.lb_qgroup != 8 && o.lb_qgroup != 16)
        return set_err(TSK_ERR_INVALID_ARG, "lb_qgroup must be 0, 1, 2, 4, 8 or 16");
    if (o.lb_both != 0 && o.lb_both != 1)
        return set_err(TSK_ERR_INVALID_ARG, "lb_both must be 0 or 1");
    if (o.raw_keys != 0 && o.raw_keys != 1)
        return set_err(TSK_ERR_INVALID_ARG, "raw_keys must be 0 or 1");
    if (o.bound_seed < 0 || o.bound_seed > 2)
        return set_err(TSK_ERR_INVALID_ARG, "bound_seed must be 0, 1 or 2");
    if (o.dtw_cascade < 0 || o.dtw_cascade > 3)
        return set_err(TSK_ERR_INVALID_ARG, "dtw_cascade must be 0, 1, 2 or 3");
    if (o.dk_box < 0 || o.dk_box > 2)
        return set_err(TSK_ERR_INVALID_ARG, "dk_box must be 0, 1 or 2");
    if (o.lb_prefix < -1 || (o.lb_prefix > 0 && (o.lb_prefix % 64 != 0 || o.lb_prefix > TSK_MAX_LEN)))
        return set_err(TSK_ERR_INVALID_ARG, "lb_prefix must be -1, 0 or a multiple of 64 up to %d",
                       TSK_MAX_LEN);
    if (o.use_graph && o.profile)
        return set_err(TSK_ERR_UNSUPPORTED, "use_graph excludes profile");
    if (fx && (o.use_graph || o.profile || o.order == TSK_ORDER_LEARNED || o.lb_both || rr ||
               stats_host))
        return set_err(TSK_ERR_UNSUPPORTED, "the fixed-workspace call excludes use_graph, "
                                            "profile, TSK_ORDER_LEARNED and lb_both");
    if (rr) {
        if (o.use_graph)
            return set_err(TSK_ERR_UNSUPPORTED, "a range query cannot run as a graph");
        o.walk_pass = 0; // its threshold is the radius: no pass may lower it
    }
    tsk_index *ix = const_cast<tsk_index *>(cix);
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    if (o.tune == TSK_TUNE_CACHED) {
        auto it = ix->tune_cache.find(tune_key(dist, band, k));
        if (it != ix->tune_cache.end())
            apply_tuned(&o, it->second);
    } else if (o.tune != TSK_TUNE_OFF) {
        return set_err(TSK_ERR_INVALID_ARG, "opts->tune %d unknown", o.tune);
    }

    QueryPlan P;
    P.D = ix->dim;
    P.dist = dist;
    P.k = k;
    P.ba = BandArgs{band.mode, band.r, band.frac};
    P.nq = n_queries;
    P.N = ix->n;
    P.chunk = chunk_queries(ix, n_queries);
    // several chunks in one graph need the per-chunk uploads of the
    // length-bucket bound (uneven-length DTW) outside it
    if (o.use_graph && P.chunk < n_queries && dist == TSK_DTW && ix->bucketed &&
        ix->min_len != ix->max_len && o.dp_kernel != 1)
        return set_err(TSK_ERR_UNSUPPORTED, "use_graph on uneven-length DTW needs the queries to "
                                            "fit one chunk (%lld here)", (long long)P.chunk);
    // the query envelope: DTW on an equal-length index, and DK there when the
    // box bound is asked for
    P.env_ok = (dist == TSK_DTW || (o.dk_box == 1 && !rr)) && ix->min_len == ix->max_len;
    // seed sizes: the greedy DK seed is a latency-bound walk (a few hundred
    // candidates give a tight threshold); the diagonal DTW seed is a cheap
    // parallel sum, so it takes more candidates.  Seeds of smallest corner
    // bound (the cascade) are likely neighbours already: 128 suffice
    // (measured on 4096 x 1M x 512 x 6: the threshold they give leaves the
    // DP work unchanged down to 128, while the walks' time halves)
    const bool plain_seedable = o.order == TSK_ORDER_PLAIN && o.bound_seed != 2;
    const bool corner_seeded =
        o.bound_seed == 1 ||
        (plain_seedable && (dist == TSK_DK || (P.env_ok && o.dtw_cascade != 2 &&
                                               o.lb_qgroup == 0 && !o.lb_both)));
    const int default_seed = corner_seeded ? 128 : (dist == TSK_DK ? 512 : 1024);
    P.seed = (int)std::min<int64_t>(ix->n, o.seed_count > 0 ? o.seed_count : default_seed);
    if (rr)
        P.seed = 0; // no threshold seeding: the radius is the threshold

    // the candidate-envelope bound: DTW on an equal-length index
    const bool lb_rev = o.lb_both && dist == TSK_DTW && P.env_ok && o.dp_kernel != 1 && !rr;
    // fixed workspace: the largest chunk whose workspace fits the region,
    // carved for the call's longest query and lent to the index for the
    // call (the index's own buffers are put back on every return)
    Workspace fixed_ws;
    struct Lend {
        tsk_index *ix;
        Workspace *w;
        bool on = false;
        ~Lend()
        {
            if (!on)
                return;
            std::swap(ix->ws, *w);
            ix->ws.h_qoff.swap(w->h_qoff);
            ix->ws.h_qtab.swap(w->h_qtab);
        }
    } lend{ix, &fixed_ws};
    if (fx) {
        int32_t qmax = 0;
        for (int64_t i = 0; i < n_queries; ++i)
            qmax = std::max<int32_t>(qmax, (int32_t)(q_offsets_host[i + 1] - q_offsets_host[i]));
        WsShape sh;
        sh.nq_total = n_queries;
        sh.k = k;
        sh.env = P.env_ok;
        sh.surv2 = P.env_ok; // DTW on equal lengths: the cascade may run
        sh.qpad = o.dp_kernel != 1;
        sh.qrows = qmax + 2 * QPAD;
        sh.qtab = dist == TSK_DTW && !P.env_ok && ix->bucketed && o.dp_kernel != 1;
        sh.qtab_floats_q = qtable_floats(qmax, pad_dim(ix->dim));
        sh.qdims_floats = ix->udim == ix->dim ? 0 : q_offsets_host[n_queries] * ix->dim;
        int64_t lo = 0, hi = P.chunk; // largest nq in [1, P.chunk] that fits
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            sh.nq = mid;
            if (carve_ws(ix, sh, nullptr, &fixed_ws) <= fx->bytes)
                lo = mid;
            else
                hi = mid - 1;
        }
        if (lo < 1) {
            sh.nq = 1;
            return set_err(TSK_ERR_INVALID_ARG,
                           "one query's workspace (%zu bytes for %lld series) exceeds the fixed "
                           "workspace of %zu bytes",
                           carve_ws(ix, sh, nullptr, &fixed_ws), (long long)ix->n, fx->bytes);
        }
        sh.nq = lo;
        P.chunk = lo;
        carve_ws(ix, sh, fx->base, &fixed_ws);
        fixed_ws.h_qoff.swap(ix->ws.h_qoff);
        fixed_ws.h_qtab.swap(ix->ws.h_qtab);
        std::swap(ix->ws, fixed_ws);
        lend.on = true;
    }
    TSK_TRY(ensure_ws(ix, P.chunk, k, P.env_ok, lb_rev, P.env_ok));
    const float *qvals = q_values_dev;
    TSK_TRY(kernel_queries(ix, q_values_dev, q_offsets_host, n_queries, s, &qvals));
    Workspace &W = ix->ws;
    if (rr)
        TSK_TRY(W.rng.ensure((size_t)P.chunk * ix->n));

    const bool profile = o.profile != 0;
    const bool timed = stats_host != nullptr || profile;
    // statistics counters only when a call reports them
    unsigned long long *const ctr = timed ? W.ctr.p : nullptr;
    if (profile) {
        // a new profile buffer starts at zero (its memory may hold anything)
        const bool fresh = ix->prof_ctr.p == nullptr;
        TSK_TRY(ix->prof_ctr.ensure(CTR_WORDS));
        if (fresh)
            fill_u64(ix->prof_ctr.p, 0ull, CTR_WORDS, s);
    }
    const size_t ev_first = ix->ev_used;

    tsk_model *model = const_cast<tsk_model *>(o.model);
    std::unique_lock<std::mutex> mlock;
    if (o.order == TSK_ORDER_LEARNED) {
        mlock = std::unique_lock<std::mutex>(model->mu);
        TSK_TRY(ix->qemb.ensure((size_t)P.chunk * model->embed));
        TSK_TRY(ix->lorder.ensure((size_t)P.chunk * ix->n));
        if (ix->emb_uid != model->uid || ix->emb_version != model->version) {
            // candidate embeddings for the model's current parameters
            TSK_TRY(ix->emb.ensure((size_t)ix->n * model->embed));
            TSK_TRY(model_embed_dev(model, ix->aos, ix->off, ix->n, ix->emb.p, s));
            ix->emb_uid = model->uid;
            ix->emb_version = model->version;
        }
    }

    // Host-side plan of one chunk of queries; prepare() does its uploads and
    // allocations, enqueue() only launches kernels (so it can be captured).
    struct Chunk {
        int64_t q0;
        int nq;
        int32_t qmin, qmax;
        const int32_t *order;
        bool lds_query, dk_split, lbu, diag_seed, dk_cascade, dtw_cascade, dtw_bseed, dk_box;
        bool surv_lb; // a second bound over the first one's survivors (surv -> surv2)
        int fast, wsel, qrows;
    };
    auto plan_chunk = [&](int64_t q0) {
        Chunk c;
        c.q0 = q0;
        c.nq = (int)std::min<int64_t>(P.chunk, n_queries - q0);
        c.order = o.order == TSK_ORDER_GIVEN ? o.order_dev + q0 * ix->n : nullptr;
        if (o.order == TSK_ORDER_LEARNED)
            c.order = ix->lorder.p;
        c.qmin = INT32_MAX;
        c.qmax = 0;
        for (int i = 0; i < c.nq; ++i) {
            const int32_t L = (int32_t)(q_offsets_host[q0 + i + 1] - q_offsets_host[q0 + i]);
            c.qmin = std::min(c.qmin, L);
            c.qmax = std::max(c.qmax, L);
        }
        c.lds_query = walk_lds_bytes(P.D, c.qmax) <= 64 * 1024 && o.dp_kernel != 1;
        c.dk_split = dist == TSK_DK && c.lds_query;
        // uneven lengths: LB_Box per length bucket, lbv by sorted position
        c.lbu = dist == TSK_DTW && !P.env_ok && ix->bucketed && o.dp_kernel != 1;
        // equal lengths: the diagonal path seeds DTW, and DK on request
        c.diag_seed = P.seed > 0 && (dist == TSK_DTW || o.dk_seed == 1) && c.qmin == c.qmax &&
                      ix->min_len == ix->max_len && ix->min_len == c.qmin && o.dp_kernel != 1;
        // threshold seed from the candidates of smallest corner bound (plain
        // order; the learned and given orders seed from their own head)
        // (DK by default in the plain order; DTW on request, or with the
        // cascade below)
        const bool seedable = !rr && P.seed > 0;
        c.dk_cascade = seedable && c.dk_split &&
                       (o.bound_seed == 1 || (o.bound_seed == 0 && o.order == TSK_ORDER_PLAIN));
        // DTW on equal lengths (by default in the plain order): the corner
        // bound first, LB_Box only for its survivors
        const bool dtw_eq = seedable && c.diag_seed && dist == TSK_DTW && P.env_ok;
        c.dtw_cascade = dtw_eq && o.lb_qgroup != 1 && !lb_rev &&
                        (o.dtw_cascade == 1 || o.dtw_cascade == 3 ||
                         (o.dtw_cascade == 0 && o.bound_seed != 2 && o.order == TSK_ORDER_PLAIN &&
                          o.lb_qgroup == 0));
        c.dtw_bseed = dtw_eq && (o.bound_seed == 1 || c.dtw_cascade);
        // DK on equal lengths, on request: the box bound of the corner survivors
        c.dk_box = c.dk_cascade && dist == TSK_DK && P.env_ok;
        // (dtw_cascade 3: the corner bound alone, no LB_Box)
        c.surv_lb = (c.dtw_cascade && o.dtw_cascade != 3) || c.dk_box;
        c.fast = pick_fast(ix, dist, band, c.qmin, c.qmax, o.dp_kernel, o.dk_band_slots, &c.wsel);
        c.qrows = c.qmax + 2 * QPAD;
        return c;
    };
    auto prepare_chunk = [&](const Chunk &c) -> int {
        if (c.lbu)
            TSK_TRY(prepare_qtables(ix, q_offsets_host, c.q0, c.nq, s));
        if (c.fast != FAST_NONE)
            TSK_TRY(W.qpad.ensure((size_t)c.nq * c.qrows * pad_dim(P.D)));
        return TSK_OK;
    };
    // 16 persistent waves per CU (4 per SIMD) hide the DP loops' load latency
    const int fast_waves = o.dp_waves_per_cu > 0 ? o.dp_waves_per_cu : 16;
    // s: the stream to enqueue on (the caller's, or the capture stream)
    auto enqueue_chunk = [&](const Chunk &c, hipEvent_t *ev, hipStream_t s) -> int {
#define TSK_MARK(i)                                                                                \
    do {                                                                                           \
        if (ev)                                                                                    \
            HIP_TRY(hipEventRecord(ev[i], s));                                                     \
    } while (0)
        const int nq = c.nq;
        const float *qv = qvals; // offsets are absolute into the query values
        W.qoff_cur = W.qoff.p + c.q0;   // every query's offsets are on the device
        TSK_MARK(0);
        fill_u32(W.tau.p, rr ? f_bits_host(rr->tau_key) : TSK_INF_BITS, nq, s);
        if (rr)
            fill_u32((uint32_t *)W.rng.p, TSK_INF_BITS, (int64_t)nq * ix->n, s);
        fill_u64(W.seedslots.p, TSK_KEY_EMPTY, (int64_t)nq * k, s);
        fill_u64(W.ubslots.p, TSK_KEY_EMPTY, (int64_t)nq * k, s);
        fill_u64(W.resslots.p, TSK_KEY_EMPTY, (int64_t)nq * k, s);
        fill_u32((uint32_t *)W.max_cnt.p, 0u, 1, s);
        fill_u32((uint32_t *)W.qcur.p, 0u, nq, s);
        fill_u64(W.work.p, 0ull, 8, s); // every task / list counter of the call
        if (o.order == TSK_ORDER_LEARNED) {
            // embed the chunk's queries, score every candidate, bucket-sort;
            // the bound pass overwrites lbv (the scores' scratch) later
            TSK_TRY(model_embed_dev(model, qv, W.qoff_cur, nq, ix->qemb.p, s));
            launch_embed_score(ix->qemb.p, nq, ix->emb.p, ix->n, model->embed, W.lbv.p, s);
            launch_bucket_order(W.lbv.p, nq, ix->n, ix->lorder.p, s);
        }
        TSK_MARK(1);
        if (P.env_ok)
            dispatch_d<EnvLaunch>(P.D, ix, qv, nq, P.ba, s);
        // survivors (lbv <= tau) of the plain candidate order, many waves per
        // query: in candidate order, or by ascending bound bucket (the first
        // cap of them)
        auto seg_compact = [&](int nqc, bool sorted, int64_t cap, unsigned long long *cctr,
                               const int32_t *order) {
            const int64_t N = ix->n;
            const int64_t nseg = (N + SEG_LEN - 1) / SEG_LEN;
            const dim3 grid((unsigned)((nseg + SEG_WAVES - 1) / SEG_WAVES), (unsigned)nqc);
            if (sorted) {
                fill_u32((uint32_t *)W.hist.p, 0u, (int64_t)nqc * SURV_BUCKETS, s);
                hipLaunchKernelGGL(k_seg_count<true>, grid, dim3(64 * SEG_WAVES), 0, s, W.lbv.p, N,
                                   nullptr, W.tau.p, W.segcnt.p, W.hist.p, cctr);
                hipLaunchKernelGGL(k_seg_bucket_scan, dim3(nqc), dim3(1024), 0, s, W.hist.p, cap,
                                   W.surv_cnt.p, W.max_cnt.p);
                hipLaunchKernelGGL(k_seg_bucket_scatter, grid, dim3(64 * SEG_WAVES), 0, s,
                                   W.lbv.p, N, W.tau.p, W.segcnt.p, W.hist.p, cap, W.surv.p);
            } else {
                hipLaunchKernelGGL(k_seg_count<false>, grid, dim3(64 * SEG_WAVES), 0, s, W.lbv.p,
                                   N, order, W.tau.p, W.segcnt.p, nullptr, cctr);
                hipLaunchKernelGGL(k_seg_scatter, grid, dim3(64 * SEG_WAVES), 0, s, W.lbv.p, N,
                                   order, W.tau.p, W.segcnt.p, W.surv.p, W.surv_cnt.p,
                                   W.max_cnt.p);
            }
        };
        SeedRingArgs seed_args{qv, W.qoff_cur, nq, c.qmax, ix->aos, ix->off, ix->len, ix->n,
                               c.order, 0, P.seed, k, P.ba, W.seedslots.p, W.tau.p, ctr,
                               nullptr, nullptr};
        const bool cascade = c.dk_cascade || c.dtw_bseed;
        if (cascade) {
            // corner bound of every pair (the threshold is still +inf: none
            // pruned), then each query's seed set = P.seed candidates of
            // small corner bound, in ascending bound
            BoundArgs cb = bound_args(ix, qv, nq, P);
            // it counts the pairs unless LB_Box still runs on all of them
            cb.ctr = (c.dk_cascade || c.dtw_cascade) ? ctr : nullptr;
            launch_corner(P.D, dist, cb, s);
            if (c.order == nullptr && 2 * P.seed <= SEEDSEG_MAX && ix->n >= 32 * (int64_t)P.seed) {
                // long lists: the smallest bound of each of 2 * seed segments,
                // the seed smallest of those (segments of equal length, none
                // empty)
                const int64_t len = (ix->n + 2 * P.seed - 1) / (2 * P.seed);
                const int nseg = (int)((ix->n + len - 1) / len);
                hipLaunchKernelGGL(k_seg_min, dim3((nseg + 3) / 4, nq), dim3(256), 0, s, W.lbv.p,
                                   ix->n, nseg, W.segkey.p);
                hipLaunchKernelGGL(k_seg_pick, dim3(nq), dim3(1024), 0, s, W.segkey.p, nseg, P.seed,
                                   ix->n, W.surv.p, W.surv_cnt.p, W.max_cnt.p);
            } else {
                // (every candidate passes the +inf threshold here: one block
                // per query counting buckets in LDS beats global atomics)
                hipLaunchKernelGGL(k_compact_sorted, dim3(nq), dim3(1024),
                                   SURV_BUCKETS * sizeof(int32_t), s, W.lbv.p, ix->n, c.order,
                                   nullptr, nullptr, W.tau.p, W.surv.p, W.surv_cnt.p,
                                   W.max_cnt.p, nullptr, (int64_t)P.seed, nullptr);
            }
            seed_args.order = W.surv.p;
        }
        if (c.diag_seed && !(c.dtw_cascade && c.lds_query)) {
            // equal lengths: diagonal-path sums seed the DTW threshold
            launch_seed_diag(P.D, dist, seed_args, s);
        } else if (P.seed > 0 && c.lds_query) {
            // (the DTW cascade: greedy walks of Alg. 1 summing their costs;
            // they follow a warped neighbour where the diagonal does not, so
            // their threshold lets the corner bound prune)
            // the first 64 candidates walk to the end and set a threshold;
            // the rest of the seed set returns early against it
            launch_seed_ring(P.D, dist, seed_args, s);
        } else {
            dispatch_d<SeedLaunch>(P.D, ix, qv, nq, P, c.order, s);
        }
        if (cascade)
            fill_u32((uint32_t *)W.max_cnt.p, 0u, 1, s); // the seed list's count
        // survivors by ascending bound by default for DTW (measured faster
        // on every class-warp workload), candidate order for DK (mixed)
        const int so = o.surv_order != 0 ? o.surv_order : (dist == TSK_DTW ? 1 : 2);
        auto compact = [&]() {
            // many waves per query for long candidate lists (one block per
            // query is latency-bound there; below 64 Ki candidates the single
            // launch costs less)
            // (a given or learned order: the unsorted variant gathers the
            // bounds through it)
            if (!c.lbu && ix->n >= (1 << 16) && (c.order == nullptr || so != 1))
                seg_compact(nq, so == 1, ix->n, ctr, c.order);
            else if (so == 1)
                hipLaunchKernelGGL(k_compact_sorted, dim3(nq), dim3(1024),
                                   SURV_BUCKETS * sizeof(int32_t), s, W.lbv.p, ix->n, c.order,
                                   c.lbu ? ix->perm : nullptr, c.lbu ? ix->inv : nullptr,
                                   W.tau.p, W.surv.p, W.surv_cnt.p, W.max_cnt.p, ctr, ix->n,
                                   nullptr);
            else
                hipLaunchKernelGGL(k_compact, dim3(nq), dim3(1024), 0, s, W.lbv.p, ix->n, c.order,
                                   c.lbu ? ix->perm : nullptr, c.lbu ? ix->inv : nullptr,
                                   W.tau.p, W.surv.p, W.surv_cnt.p, W.max_cnt.p, ctr);
        };
        if (c.surv_lb)
            compact(); // the corner survivors, before LB_Box or the DK box bound
        TSK_MARK(2);
        BoundArgs ba = bound_args(ix, qv, nq, P);
        ba.ctr = ctr;
        if (rr)
            ba.ubslots = nullptr;
        if (c.surv_lb) {
            // LB_Box (DTW) or the DK box bound of the corner survivors only
            // (lbv: their bound or +inf)
            // (default: a prefix of 64 points when the banded lane-per-pair
            // DP follows; measured on 1024 x 1M x 512 x 6 the bound stage
            // falls 13.4 -> 4.7 ms and the pairs it prunes 1.0188803e9 ->
            // 1.018880e9, the DP work unchanged.  Before the general DP the
            // survivors' order by their full bound matters more: unbanded
            // DTW on 256 x 100 000 x 128 x 3 took 13.5 ms with the prefix,
            // 7.3 ms without)
            const int def_prefix = c.fast == FAST_BAND ? 64 : 0;
            ba.lb_prefix = dist == TSK_DTW ? (o.lb_prefix == 0 ? def_prefix : std::max(0, o.lb_prefix))
                                           : 0;
            launch_bound_lb_surv(P.D, dist, ba, W.surv.p, W.surv_cnt.p, W.max_cnt.p,
                                 W.work.p + 6, ix->n_cu * 8, s);
        } else if (c.dk_cascade || c.dtw_cascade) {
            // the corner bounds are in lbv already
        } else if (c.dk_split) {
            launch_corner(P.D, dist, ba, s);
        } else if (dist == TSK_DTW && P.env_ok && o.dp_kernel != 1) {
            if (o.lb_qgroup == 1 && lb_pp_lds_bytes(P.D, ba.env_n) <= LB_PP_MAX_LDS) {
                launch_bound_lb_pp(P.D, ba, s); // per pair, early abandoning
            } else {
                // 16 queries per candidate load when asked for, or by default
                // once the database outgrows the 256 MB MALL
                const bool big = (int64_t)ix->total * ix->dim * 4 > ((int64_t)256 << 20);
                ba.qgroup = (o.lb_qgroup == 16 || (o.lb_qgroup == 0 && big)) ? 16 : 8;
                launch_bound_lb(P.D, ba, false, s);
            }
        } else if (c.lbu) {
            launch_qtable(P.D, qv, W.qoff_cur, nq, W.qtab_off.p, W.qtab.p, s);
            launch_bound_lbu(P.D, ba, bucket_args(ix), W.qtab.p, W.qtab_off.p,
                             o.lb_qgroup > 1 ? std::min(o.lb_qgroup, 8) : 4, false, s);
        } else {
            dispatch_d<BoundLaunch>(P.D, ba, dist, false, s);
        }
        TSK_MARK(3);
        if (c.surv_lb) {
            // the corner survivors re-ranked by their second bound (into surv2)
            fill_u32((uint32_t *)W.max_cnt.p, 0u, 1, s);
            hipLaunchKernelGGL(k_compact_sorted, dim3(nq), dim3(1024),
                               SURV_BUCKETS * sizeof(int32_t), s, W.lbv.p, ix->n, W.surv.p,
                               nullptr, nullptr, W.tau.p, W.surv2.p, W.surv_cnt.p, W.max_cnt.p,
                               ctr, ix->n, W.surv_cnt.p);
        } else {
            compact();
        }
        int32_t *const surv_dp = c.surv_lb ? W.surv2.p : W.surv.p;
        if (lb_rev) {
            // LB_Box in both orientations: the survivors' bounds become the
            // larger one (queries of another length keep theirs)
            launch_bound_lb_rev(P.D, ix->aos, ix->off, ix->n, ix->max_len, P.ba, W.cenv.p, qv,
                                W.qoff_cur, nq, W.surv.p, W.surv_cnt.p, W.lbv.p, s);
        }
        // the greedy pass over the corner survivors costs more than the DP
        // work its tighter threshold saves on the class-warp workloads, so
        // it runs only on request
        if (c.dk_split && o.walk_pass == 1) {
            // greedy bound (Alg. 1) of every survivor of the corner bound
            FastArgs wa = fast_args(ix, nq, P, 0);
            wa.ctr = ctr;
            wa.work = W.work.p + 4;
            launch_walk_dk(P.D, wa, qv, W.ubslots.p, ix->n_cu * 8, c.qmax, s);
        }
        TSK_MARK(4);
        DpArgs da = dp_args(ix, qv, nq, P);
        da.ctr = ctr;
        da.surv = surv_dp;
        da.lb_inv = c.lbu ? ix->inv : nullptr;
        da.range_out = rr ? W.rng.p : nullptr;
        if (o.dp_rows != 0)
            da.rows_per_lane = o.dp_rows;
        if (c.fast != FAST_NONE) {
            dispatch_d<QpadLaunch>(P.D, qv, W.qoff_cur, nq, c.qrows, W.qpad.p, s);
            TSK_MARK(5);
            FastArgs fa = fast_args(ix, nq, P, c.qrows);
            fa.ctr = ctr;
            fa.surv = surv_dp;
            fa.lb_inv = c.lbu ? ix->inv : nullptr;
            fa.range_out = rr ? W.rng.p : nullptr;
            if (c.fast == FAST_TUBE32) {
                // survivors per wave task: larger databases leave more
                // survivors per query, and larger tasks then cut the lanes'
                // idle tails at task ends (measured: 256 best on 1M series,
                // 64 on 20 000)
                fa.task = o.task_size > 0 ? o.task_size
                                          : (ix->n >= (1 << 19) ? 256 : ix->n >= (1 << 16) ? 128 : 64);
                // 16-row windows: the live tube of near neighbours is a few
                // rows wide; the rare wider ones finish in the general DP
                const bool equal = c.qmin == c.qmax && ix->min_len == ix->max_len && ix->min_len == c.qmin;
                launch_tube(P.D, fa, o.tube_rows == 0 ? 16 : o.tube_rows, equal, ix->n_cu * fast_waves,
                            c.qmax, s);
            } else {
                fa.dk_virtual = c.fast == FAST_BAND_DKV ? 1 : 0;
                launch_band(P.D, dist, c.wsel, fa, ix->n_cu * fast_waves, s);
            }
            TSK_MARK(6);
            da.work = W.work.p + 2;
            launch_dp_wave(P.D, dist, DPW_FALLBACK, da, dp_blocks(ix), s);
        } else {
            TSK_MARK(5);
            TSK_MARK(6);
            launch_dp_wave(P.D, dist, DPW_SURV, da, dp_blocks(ix), s);
        }
        TSK_MARK(7);
        if (rr)
            hipLaunchKernelGGL(k_range_count, dim3(nq), dim3(256), 0, s, W.rng.p, ix->n,
                               W.rcnt.p);
        else if (dist == TSK_DK && !o.raw_keys)
            hipLaunchKernelGGL(k_finalize<DIST_DK>, dim3(nq), dim3(64), 0, s, W.resslots.p, nq, k,
                               out_ids_dev + c.q0 * k, out_dist_dev + c.q0 * k);
        else
            hipLaunchKernelGGL(k_finalize<DIST_DTW>, dim3(nq), dim3(64), 0, s, W.resslots.p, nq,
                               k, out_ids_dev + c.q0 * k, out_dist_dev + c.q0 * k);
        TSK_MARK(8);
#undef TSK_MARK
        HIP_TRY(hipGetLastError());
        return TSK_OK;
    };

    if (o.cancel_flag_host && *o.cancel_flag_host != 0)
        return set_err(TSK_ERR_CANCELLED, "cancelled before any device work");
    // every query's offsets to the device once (the chunks index into them)
    TSK_TRY(W.qoff.ensure(n_queries + 1));
    TSK_TRY(upload_qoff(ix, q_offsets_host, 0, n_queries, s));
    if (o.use_graph) {
        // every chunk of the call in one graph, replayed from a cached
        // executable graph when the call repeats (same inputs, outputs,
        // shape and options).  Buffers are sized for the largest chunk first,
        // so no chunk's preparation reallocates one the capture addressed.
        std::vector<Chunk> chunks;
        for (int64_t q0 = 0; q0 < n_queries; q0 += P.chunk)
            chunks.push_back(plan_chunk(q0));
        int qrows_max = 0;
        for (const Chunk &c : chunks)
            qrows_max = std::max(qrows_max, c.fast != FAST_NONE ? c.qrows : 0);
        if (qrows_max > 0)
            TSK_TRY(W.qpad.ensure((size_t)P.chunk * qrows_max * pad_dim(P.D)));
        for (const Chunk &c : chunks)
            TSK_TRY(prepare_chunk(c));
        if (o.order == TSK_ORDER_LEARNED)
            TSK_TRY(model_reserve_rows(model, std::min<int64_t>(P.chunk, EMBED_CHUNK)));
        std::vector<int64_t> key = {(int64_t)(uintptr_t)q_values_dev, n_queries, k, dist,
                                    band.mode, band.r, (int64_t)f_bits_host(band.frac),
                                    (int64_t)(uintptr_t)out_ids_dev,
                                    (int64_t)(uintptr_t)out_dist_dev, (int64_t)(uintptr_t)s,
                                    o.order, (int64_t)(uintptr_t)o.order_dev, o.seed_count,
                                    o.dp_kernel, o.walk_pass, o.task_size, o.tube_rows,
                                    o.lb_qgroup, o.dk_band_slots, o.surv_order, o.dp_rows,
                                    o.dp_waves_per_cu, o.dk_seed, o.lb_both, o.raw_keys,
                                    o.bound_seed, o.dtw_cascade, o.dk_box, o.lb_prefix,
                                    (int64_t)timed};
        // every workspace buffer the captured kernels address: a buffer
        // reallocated by another call changes the key
        for (const void *ptr :
             {(const void *)W.tau.p, (const void *)W.seedslots.p, (const void *)W.ubslots.p,
              (const void *)W.resslots.p, (const void *)W.lbv.p, (const void *)W.surv.p,
              (const void *)W.segcnt.p, (const void *)W.hist.p, (const void *)W.segkey.p,
              (const void *)W.surv_cnt.p, (const void *)W.max_cnt.p, (const void *)W.ctr.p,
              (const void *)W.qcur.p,
              (const void *)W.work.p, (const void *)W.qoff.p, (const void *)W.env.p,
              (const void *)W.tbuf.p, (const void *)W.qpad.p, (const void *)W.fb.p,
              (const void *)W.qtab.p, (const void *)W.qtab_off.p, (const void *)W.cenv.p,
              (const void *)W.surv2.p, (const void *)qvals, (const void *)o.model,
              (const void *)ix->emb.p,
              (const void *)ix->qemb.p, (const void *)ix->lorder.p,
              (const void *)(model ? model->x.p : nullptr),
              (const void *)(model ? model->a1.p : nullptr),
              (const void *)(model ? model->a2.p : nullptr),
              (const void *)(model ? model->params.p : nullptr)})
            key.push_back((int64_t)(uintptr_t)ptr);
        key.insert(key.end(), q_offsets_host, q_offsets_host + n_queries + 1);
        if (stats_host) {
            if (!ix->gev[0])
                for (auto &e : ix->gev)
                    HIP_TRY(hipEventCreate(&e));
            HIP_TRY(hipEventRecord(ix->gev[0], s));
        }
        if (!ix->graph_exec || key != ix->graph_key) {
            if (ix->graph_exec) {
                (void)hipGraphExecDestroy(ix->graph_exec);
                ix->graph_exec = nullptr;
            }
            // captured on a private stream (the caller's may be the null
            // stream, which cannot be captured); launched on the caller's
            if (!ix->cap_stream)
                HIP_TRY(hipStreamCreateWithFlags(&ix->cap_stream, hipStreamNonBlocking));
            hipStream_t cs = ix->cap_stream;
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            fill_u64(W.ctr.p, 0ull, CTR_WORDS, cs);
            int rc = TSK_OK;
            for (const Chunk &c : chunks)
                if (rc == TSK_OK)
                    rc = enqueue_chunk(c, nullptr, cs);
            const hipError_t ec = hipStreamEndCapture(cs, &g);
            if (rc != TSK_OK) {
                if (g)
                    (void)hipGraphDestroy(g);
                return rc;
            }
            HIP_TRY(ec);
            const hipError_t ei = hipGraphInstantiate(&ix->graph_exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIP_TRY(ei);
            ix->graph_key = key;
            ++ix->graph_builds;
        }
        HIP_TRY(hipGraphLaunch(ix->graph_exec, s));
        if (stats_host)
            HIP_TRY(hipEventRecord(ix->gev[1], s));
    } else {
        fill_u64(W.ctr.p, 0ull, CTR_WORDS, s);
        for (int64_t q0 = 0; q0 < n_queries; q0 += P.chunk) {
            if (o.cancel_flag_host && *o.cancel_flag_host != 0)
                return set_err(TSK_ERR_CANCELLED, "cancelled before query %lld", (long long)q0);
            const Chunk c = plan_chunk(q0);
            TSK_TRY(prepare_chunk(c));
            hipEvent_t *ev = nullptr;
            if (timed)
                TSK_TRY(take_events(ix, &ev));
            TSK_TRY(enqueue_chunk(c, ev, s));
            if (rr) {
                // counts to the host, then this chunk's hits in id order
                std::vector<int64_t> cnt(c.nq);
                HIP_TRY(hipMemcpyAsync(cnt.data(), W.rcnt.p, c.nq * sizeof(int64_t),
                                       hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                std::vector<int64_t> qo(c.nq + 1);
                qo[0] = rr->offsets_host[c.q0];
                for (int i = 0; i < c.nq; ++i)
                    qo[i + 1] = qo[i] + cnt[i];
                for (int i = 0; i < c.nq; ++i)
                    rr->offsets_host[c.q0 + i + 1] = qo[i + 1];
                if (qo[c.nq] <= rr->capacity && qo[c.nq] > qo[0]) {
                    TSK_TRY(W.rqoff.ensure(c.nq + 1));
                    HIP_TRY(hipMemcpyAsync(W.rqoff.p, qo.data(), (c.nq + 1) * sizeof(int64_t),
                                           hipMemcpyHostToDevice, s));
                    if (dist == TSK_DK)
                        hipLaunchKernelGGL(k_range_fill<DIST_DK>, dim3(c.nq), dim3(256), 0, s,
                                           W.rng.p, ix->n, W.rqoff.p, rr->ids, rr->dist);
                    else
                        hipLaunchKernelGGL(k_range_fill<DIST_DTW>, dim3(c.nq), dim3(256), 0, s,
                                           W.rng.p, ix->n, W.rqoff.p, rr->ids, rr->dist);
                    HIP_TRY(hipGetLastError());
                    // the offsets upload reads qo: finish before it goes away
                    HIP_TRY(hipStreamSynchronize(s));
                }
            }
        }
    }
    HIP_TRY(hipGetLastError());
    if (profile) {
        hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(256), 0, s, ix->prof_ctr.p, W.ctr.p,
                           (int)CTR_WORDS);
        ix->prof_calls += 1;
        ix->prof_chunks += (n_queries + P.chunk - 1) / P.chunk;
    }
    if (stats_host) {
        unsigned long long words[CTR_WORDS], c[C_NUM];
        HIP_TRY(hipMemcpyAsync(words, W.ctr.p, sizeof(words), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        ctr_sum(words, c);
        memset(stats_host, 0, sizeof(*stats_host));
        stats_from(stats_host, c);
        stats_host->calls = 1;
        stats_host->chunks = (n_queries + P.chunk - 1) / P.chunk;
        if (o.use_graph) {
            // a replayed graph is timed as one interval (no stage marks)
            HIP_TRY(hipEventElapsedTime(&stats_host->ms_total, ix->gev[0], ix->gev[1]));
        } else {
            float t[NEV - 1];
            TSK_TRY(sum_events(ix, ev_first, ix->ev_used, t));
            if (!profile)
                ix->ev_used = ev_first; // these events are not part of a profile
            stats_times(stats_host, t);
        }
    }
    return TSK_OK;
}

extern "C" int tsk_knn_query(const tsk_index *cix, const float *q_values_dev,
                             const int64_t *q_offsets_host, int64_t n_queries, int32_t k,
                             int32_t dist, tsk_band band, const tsk_query_opts *opts,
                             int64_t *out_ids_dev, float *out_dist_dev, tsk_stats *stats_host,
                             void *hip_stream)
{
    return scan_impl(cix, q_values_dev, q_offsets_host, n_queries, k, dist, band, opts,
                     out_ids_dev, out_dist_dev, stats_host, hip_stream, nullptr);
}

extern "C" int tsk_knn_query_noalloc(const tsk_index *cix, const float *q_values_dev,
                                     const int64_t *q_offsets_host, int64_t n_queries, int32_t k,
                                     int32_t dist, tsk_band band, const tsk_query_opts *opts,
                                     int64_t *out_ids_dev, float *out_dist_dev, void *hip_stream)
{
    g_err.clear();
    if (!cix)
        return set_err(TSK_ERR_INVALID_ARG, "index is NULL");
    TSK_TRY(check_device(cix));
    FixedWs fx;
    TSK_TRY(scratch_address(cix->device, &fx.base));
    fx.bytes = (size_t)TSK_NOALLOC_SCRATCH_BYTES;
    return scan_impl(cix, q_values_dev, q_offsets_host, n_queries, k, dist, band, opts,
                     out_ids_dev, out_dist_dev, nullptr, hip_stream, nullptr, &fx);
}

// Largest fp32 key whose reported distance is within the radius: DTW keys
// are distances; a DK key's distance is its correctly rounded sqrt, which
// is monotone, so the set of keys within the radius is a prefix.  The fp32
// sqrt is taken through double (exact square root rounded twice, which is
// the correctly rounded fp32 value) and neighbours by stepping bit patterns.
static bool sqrt_within(float key, float radius)
{
    return (float)std::sqrt((double)key) <= radius;
}

static float step_bits(float x, int d)
{
    uint32_t u;
    memcpy(&u, &x, sizeof(u));
    u = (uint32_t)((int64_t)u + d);
    memcpy(&x, &u, sizeof(u));
    return x;
}

static float range_key(int32_t dist, float radius)
{
    if (dist == TSK_DTW)
        return radius;
    if (std::isinf(radius))
        return radius;
    float t = (float)((double)radius * (double)radius);
    while (!std::isinf(step_bits(t, 1)) && sqrt_within(step_bits(t, 1), radius))
        t = step_bits(t, 1);
    while (t > 0.0f && !sqrt_within(t, radius))
        t = step_bits(t, -1);
    return t;
}

extern "C" int tsk_range_query(const tsk_index *cix, const float *q_values_dev,
                               const int64_t *q_offsets_host, int64_t n_queries, double radius_d,
                               int32_t dist, const tsk_band *band_p, const tsk_query_opts *opts,
                               int64_t capacity, int64_t *out_ids_dev, float *out_dist_dev,
                               int64_t *out_offsets_host, tsk_stats *stats_host,
                               void *hip_stream)
{
    g_err.clear();
    if (!(radius_d >= 0.0)) // also rejects NaN
        return set_err(TSK_ERR_INVALID_ARG, "radius must be >= 0");
    // distances are fp32: a hit is a series whose fp32 distance is <= the
    // radius rounded down to fp32
    float radius = (float)radius_d;
    if ((double)radius > radius_d)
        radius = step_bits(radius, -1);
    tsk_band band;
    memset(&band, 0, sizeof(band));
    band.mode = TSK_BAND_NONE;
    if (band_p)
        band = *band_p;
    if (!out_offsets_host)
        return set_err(TSK_ERR_INVALID_ARG, "out_offsets_host is NULL");
    if (capacity < 0 || (capacity > 0 && (!out_ids_dev || !out_dist_dev)))
        return set_err(TSK_ERR_INVALID_ARG, "capacity < 0, or output pointers NULL");
    if (n_queries >= 1)
        out_offsets_host[0] = 0;
    RangeReq rr{range_key(dist, radius), capacity, out_ids_dev, out_dist_dev, out_offsets_host};
    TSK_TRY(scan_impl(cix, q_values_dev, q_offsets_host, n_queries, 1, dist, band, opts, nullptr,
                      nullptr, stats_host, hip_stream, &rr));
    if (out_offsets_host[n_queries] > capacity)
        return set_err(TSK_ERR_INVALID_ARG,
                       "%lld hits do not fit the capacity of %lld (offsets are filled)",
                       (long long)out_offsets_host[n_queries], (long long)capacity);
    return TSK_OK;
}

extern "C" int tsk_index_profile(tsk_index *ix, tsk_stats *out, int32_t reset)
{
    g_err.clear();
    if (!ix || !out)
        return set_err(TSK_ERR_INVALID_ARG, "index and out must be non-NULL");
    std::lock_guard<std::mutex> lock(ix->mu);
    memset(out, 0, sizeof(*out));
    float t[NEV - 1];
    TSK_TRY(sum_events(ix, 0, ix->ev_used, t));
    if (ix->prof_ctr.p) {
        unsigned long long words[CTR_WORDS], c[C_NUM];
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(words, ix->prof_ctr.p, sizeof(words), hipMemcpyDeviceToHost));
        ctr_sum(words, c);
        stats_from(out, c);
    }
    out->calls = ix->prof_calls;
    out->chunks = ix->prof_chunks;
    stats_times(out, t);
    if (reset) {
        ix->ev_used = 0;
        ix->prof_calls = 0;
        ix->prof_chunks = 0;
        if (ix->prof_ctr.p) {
            fill_u64(ix->prof_ctr.p, 0ull, CTR_WORDS, nullptr);
            HIP_TRY(hipDeviceSynchronize());
        }
    }
    return TSK_OK;
}

// DK distances from squared DK keys (the output rounding of k_finalize).
static __global__ void k_sqrt_keys(const float *__restrict__ keys, float *__restrict__ out,
                                   int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = sqrt_rn_f32(keys[i]);
}

extern "C" int tsk_dk_distances(const float *keys_dev, float *out_dev, int64_t n,
                                void *hip_stream)
{
    g_err.clear();
    if (n < 0 || (n > 0 && (!keys_dev || !out_dev)))
        return set_err(TSK_ERR_INVALID_ARG, "n must be >= 0 and the pointers non-NULL");
    if (n == 0)
        return TSK_OK;
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    TSK_TRY(check_dev_ptr(keys_dev, dev, "keys_dev"));
    TSK_TRY(check_dev_ptr(out_dev, dev, "out_dev"));
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_sqrt_keys, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, keys_dev,
                       out_dev, n);
    HIP_TRY(hipGetLastError());
    return TSK_OK;
}

extern "C" int tsk_pair_distances(const tsk_index *cix, const float *q_values_dev,
                                  const int64_t *q_offsets_host, int64_t n_queries, int32_t dist,
                                  tsk_band band, float *out_keys_dev, void *hip_stream)
{
    g_err.clear();
    TSK_TRY(check_queries(cix, q_values_dev, q_offsets_host, n_queries, dist, band));
    if (!out_keys_dev)
        return set_err(TSK_ERR_INVALID_ARG, "out_keys_dev is NULL");
    TSK_TRY(check_dev_ptr(out_keys_dev, cix->device, "out_keys_dev"));
    tsk_index *ix = const_cast<tsk_index *>(cix);
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    QueryPlan P;
    memset(&P, 0, sizeof(P));
    P.D = ix->dim;
    P.dist = dist;
    P.k = 1;
    P.ba = BandArgs{band.mode, band.r, band.frac};
    const int64_t chunk = chunk_queries(ix, n_queries);
    TSK_TRY(ensure_ws(ix, chunk, 1, false));
    const float *qvals = q_values_dev;
    TSK_TRY(kernel_queries(ix, q_values_dev, q_offsets_host, n_queries, s, &qvals));
    for (int64_t q0 = 0; q0 < n_queries; q0 += chunk) {
        const int nq = (int)std::min<int64_t>(chunk, n_queries - q0);
        TSK_TRY(upload_qoff(ix, q_offsets_host, q0, nq, s));
        fill_u64(ix->ws.work.p, 0ull, 8, s);
        fill_u64(ix->ws.ctr.p, 0ull, CTR_WORDS, s);
        DpArgs da = dp_args(ix, qvals, nq, P);
        da.out_all = out_keys_dev + q0 * ix->n;
        launch_dp_wave(P.D, dist, DPW_ALLPAIRS, da, dp_blocks(ix), s);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(s));
    return TSK_OK;
}

extern "C" int tsk_pair_bounds(const tsk_index *cix, const float *q_values_dev,
                               const int64_t *q_offsets_host, int64_t n_queries, int32_t dist,
                               tsk_band band, float *out_lb_dev, float *out_ub_dev,
                               int32_t *out_steps_dev, void *hip_stream)
{
    g_err.clear();
    TSK_TRY(check_queries(cix, q_values_dev, q_offsets_host, n_queries, dist, band));
    TSK_TRY(check_dev_ptr(out_lb_dev, cix->device, "out_lb_dev"));
    TSK_TRY(check_dev_ptr(out_ub_dev, cix->device, "out_ub_dev"));
    TSK_TRY(check_dev_ptr(out_steps_dev, cix->device, "out_steps_dev"));
    tsk_index *ix = const_cast<tsk_index *>(cix);
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    QueryPlan P;
    memset(&P, 0, sizeof(P));
    P.D = ix->dim;
    P.dist = dist;
    P.k = 1;
    P.ba = BandArgs{band.mode, band.r, band.frac};
    P.env_ok = (dist == TSK_DTW) && ix->min_len == ix->max_len;
    const int64_t chunk = chunk_queries(ix, n_queries);
    TSK_TRY(ensure_ws(ix, chunk, 1, P.env_ok));
    const float *qvals = q_values_dev;
    TSK_TRY(kernel_queries(ix, q_values_dev, q_offsets_host, n_queries, s, &qvals));
    for (int64_t q0 = 0; q0 < n_queries; q0 += chunk) {
        const int nq = (int)std::min<int64_t>(chunk, n_queries - q0);
        TSK_TRY(upload_qoff(ix, q_offsets_host, q0, nq, s));
        fill_u64(ix->ws.ctr.p, 0ull, CTR_WORDS, s);
        if (P.env_ok)
            dispatch_d<EnvLaunch>(P.D, ix, qvals, nq, P.ba, s);
        BoundArgs ba = bound_args(ix, qvals, nq, P);
        ba.dbg_lb = out_lb_dev ? out_lb_dev + q0 * ix->n : nullptr;
        ba.dbg_ub = out_ub_dev ? out_ub_dev + q0 * ix->n : nullptr;
        ba.dbg_steps = out_steps_dev ? out_steps_dev + q0 * ix->n : nullptr;
        // the k-NN path's kernels where they apply (LB_Box of equal-length
        // indexes, LDS walks), the general bound kernel for the rest
        dispatch_d<BoundLaunch>(P.D, ba, dist, true, s);
        if (dist == TSK_DTW && P.env_ok && ba.dbg_lb)
            launch_bound_lb(P.D, ba, true, s);
        if (dist == TSK_DTW && !P.env_ok && ix->bucketed && ba.dbg_lb) {
            TSK_TRY(prepare_qtables(ix, q_offsets_host, q0, nq, s));
            launch_qtable(P.D, qvals, ix->ws.qoff.p, nq, ix->ws.qtab_off.p, ix->ws.qtab.p, s);
            launch_bound_lbu(P.D, ba, bucket_args(ix), ix->ws.qtab.p, ix->ws.qtab_off.p, 4, true, s);
        }
        int32_t qmax = 0;
        for (int i = 0; i < nq; ++i)
            qmax = std::max<int32_t>(qmax, (int32_t)(q_offsets_host[q0 + i + 1] - q_offsets_host[q0 + i]));
        if (ba.dbg_ub && ba.dbg_steps && walk_lds_bytes(P.D, qmax) <= 64 * 1024) {
            SeedRingArgs r{qvals, ix->ws.qoff.p, nq, qmax, ix->aos, ix->off, ix->len, ix->n,
                           nullptr, 0, (int)std::min<int64_t>(ix->n, INT32_MAX), 1, P.ba,
                           ix->ws.seedslots.p, ix->ws.tau.p, ix->ws.ctr.p, ba.dbg_ub, ba.dbg_steps};
            launch_seed_ring(P.D, dist, r, s);
        }
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(s));
    return TSK_OK;
}

extern "C" int tsk_pair_dk_box(const tsk_index *cix, const float *q_values_dev,
                               const int64_t *q_offsets_host, int64_t n_queries, tsk_band band,
                               float *out_dev, void *hip_stream)
{
    g_err.clear();
    TSK_TRY(check_queries(cix, q_values_dev, q_offsets_host, n_queries, TSK_DK, band));
    if (!out_dev)
        return set_err(TSK_ERR_INVALID_ARG, "out_dev is NULL");
    TSK_TRY(check_dev_ptr(out_dev, cix->device, "out_dev"));
    if (cix->min_len != cix->max_len)
        return set_err(TSK_ERR_UNSUPPORTED, "the DK box bound needs series of one length "
                                            "(index lengths %d .. %d)", cix->min_len, cix->max_len);
    tsk_index *ix = const_cast<tsk_index *>(cix);
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    QueryPlan P;
    memset(&P, 0, sizeof(P));
    P.D = ix->dim;
    P.dist = TSK_DK;
    P.k = 1;
    P.ba = BandArgs{band.mode, band.r, band.frac};
    P.env_ok = true;
    const int64_t chunk = chunk_queries(ix, n_queries);
    TSK_TRY(ensure_ws(ix, chunk, 1, true));
    const float *qvals = q_values_dev;
    TSK_TRY(kernel_queries(ix, q_values_dev, q_offsets_host, n_queries, s, &qvals));
    Workspace &W = ix->ws;
    const int64_t N = ix->n;
    for (int64_t q0 = 0; q0 < n_queries; q0 += chunk) {
        const int nq = (int)std::min<int64_t>(chunk, n_queries - q0);
        TSK_TRY(upload_qoff(ix, q_offsets_host, q0, nq, s));
        fill_u64(W.ctr.p, 0ull, CTR_WORDS, s);
        dispatch_d<EnvLaunch>(P.D, ix, qvals, nq, P.ba, s);
        // every candidate is a survivor; no threshold
        hipLaunchKernelGGL(k_iota_rows, dim3(grid_for(nq * N, 256, 8192)), dim3(256), 0, s,
                           W.surv.p, (int64_t)nq, N);
        fill_u32((uint32_t *)W.surv_cnt.p, (uint32_t)N, nq, s);
        fill_u32((uint32_t *)W.max_cnt.p, (uint32_t)N, 1, s);
        fill_u32(W.tau.p, TSK_INF_BITS, nq, s);
        fill_u64(W.work.p, 0ull, 8, s);
        BoundArgs ba = bound_args(ix, qvals, nq, P);
        ba.lbv = out_dev + q0 * N;
        launch_bound_lb_surv(P.D, TSK_DK, ba, W.surv.p, W.surv_cnt.p, W.max_cnt.p, W.work.p + 6,
                             ix->n_cu * 8, s);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(s));
    return TSK_OK;
}

extern "C" int tsk_tune(tsk_index *ix, const float *q_values_dev, const int64_t *q_offsets_host,
                        int64_t n_queries, int32_t k, int32_t dist, tsk_band band,
                        const tsk_query_opts *base, const tsk_tune_opts *topts,
                        tsk_query_opts *best_out, float *best_ms_out, void *hip_stream)
{
    g_err.clear();
    TSK_TRY(check_queries(ix, q_values_dev, q_offsets_host, n_queries, dist, band));
    if (k < 1 || k > TSK_MAX_K)
        return set_err(k < 1 ? TSK_ERR_INVALID_ARG : TSK_ERR_UNSUPPORTED, "k %d out of range", k);
    if (topts && topts->size != (int64_t)sizeof(tsk_tune_opts))
        return set_err(TSK_ERR_INVALID_ARG, "tune_opts->size mismatch");
    tsk_query_opts b;
    memset(&b, 0, sizeof(b));
    b.size = sizeof(b);
    b.walk_pass = -1;
    if (base) {
        if (base->size != (int64_t)sizeof(tsk_query_opts))
            return set_err(TSK_ERR_INVALID_ARG, "base->size mismatch");
        b = *base;
    }
    b.profile = 0;
    b.use_graph = 0;
    b.tune = TSK_TUNE_OFF;
    const int64_t S = std::min<int64_t>(n_queries, topts && topts->sample_queries > 0
                                                      ? topts->sample_queries : 64);
    const int reps = topts && topts->reps > 0 ? topts->reps : 2;
    hipStream_t s = (hipStream_t)hip_stream;
    DevBuf<int64_t> ids;
    DevBuf<float> dd;
    TSK_TRY(ids.ensure(S * k));
    TSK_TRY(dd.ensure(S * k));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    std::vector<int64_t> first, got(S * k);
    int trials = 0;
    // best of `reps` timed calls after one untimed call; rows must not change
    auto trial = [&](const tsk_query_opts &o, float *ms) -> int {
        *ms = INFINITY;
        for (int r = 0; r <= reps; ++r) {
            HIP_TRY(hipEventRecord(e0, s));
            TSK_TRY(tsk_knn_query(ix, q_values_dev, q_offsets_host, S, k, dist, band, &o, ids.p,
                                  dd.p, nullptr, s));
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float t = 0.0f;
            HIP_TRY(hipEventElapsedTime(&t, e0, e1));
            if (r > 0)
                *ms = std::min(*ms, t);
        }
        HIP_TRY(hipMemcpy(got.data(), ids.p, got.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
        if (first.empty())
            first = got;
        else if (got != first)
            return set_err(TSK_ERR_DEVICE, "tuning trial %d changed the k-NN rows", trials);
        ++trials;
        return TSK_OK;
    };
    auto run = [&]() -> int {
        const bool dk_free = dist == TSK_DK && band.mode == TSK_BAND_NONE;
        const bool lbu = dist == TSK_DTW && ix->bucketed;
        struct Knob {
            int32_t tsk_query_opts::*field;
            std::vector<int32_t> values;
        };
        std::vector<Knob> knobs;
        std::vector<int32_t> seeds;
        for (int32_t v : {128, 256, 512, 1024, 2048, 4096})
            if (v <= ix->n)
                seeds.push_back(v);
        knobs.push_back({&tsk_query_opts::seed_count, seeds});
        if (dk_free && ix->min_len == ix->max_len) {
            knobs.push_back({&tsk_query_opts::dk_seed, {1}});
            knobs.push_back({&tsk_query_opts::dk_band_slots, {32, 56, 104, 128}});
        }
        if (dk_free) {
            knobs.push_back({&tsk_query_opts::tube_rows, {8, 16, 32}});
            knobs.push_back({&tsk_query_opts::task_size, {32, 64, 128, 256}});
            knobs.push_back({&tsk_query_opts::walk_pass, {0, 1}});
        }
        if (lbu)
            knobs.push_back({&tsk_query_opts::lb_qgroup, {2, 4, 8}});
        else if (dist == TSK_DTW) {
            knobs.push_back({&tsk_query_opts::dtw_cascade, {1, 2}}); // corner first or not
            knobs.push_back({&tsk_query_opts::lb_qgroup, {1, 8, 16}}); // LB kernel and query group
        }
        if (dk_free)
            knobs.push_back({&tsk_query_opts::bound_seed, {1, 2}});
        knobs.push_back({&tsk_query_opts::surv_order, {1, 2}});
        knobs.push_back({&tsk_query_opts::dp_rows, {1, 2, 4}});
        knobs.push_back({&tsk_query_opts::dp_waves_per_cu, {8, 16, 32}});
        tsk_query_opts cur = b;
        float cur_ms = 0.0f;
        TSK_TRY(trial(cur, &cur_ms));
        for (const Knob &kn : knobs) {
            for (int32_t v : kn.values) {
                if (cur.*(kn.field) == v)
                    continue;
                tsk_query_opts t = cur;
                t.*(kn.field) = v;
                float ms = 0.0f;
                TSK_TRY(trial(t, &ms));
                if (ms < 0.98f * cur_ms) { // a clear gain only
                    cur = t;
                    cur_ms = ms;
                }
            }
        }
        {
            std::lock_guard<std::mutex> lock(ix->mu);
            ix->tune_cache[tune_key(dist, band, k)] = cur;
        }
        if (best_out)
            *best_out = cur;
        if (best_ms_out)
            *best_ms_out = cur_ms;
        return TSK_OK;
    };
    const int rc = run();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
