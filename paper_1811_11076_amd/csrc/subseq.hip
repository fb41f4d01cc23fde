// Subsequence search entry point (tsk_subseq_query): the long series are
// taken as they are (AoS on the device), with no index.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "kernels_sub.hpp"
#include "runtime.hpp"
#include "tsknn.h"

using namespace tsk;

static_assert(TSK_SUB_MAX_QLEN == SUB_MAX_QLEN, "query length limit");

namespace {

template <int D, int R> void sub_dp_launch(const SubArgs &a, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_sub_dp<D, R>), dim3(blocks), dim3(256), 0, s, a);
}

template <int D, int R> void sub_start_launch(const SubArgs &a, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_sub_start<D, R>), dim3(blocks), dim3(256), 0, s, a);
}

template <int D> void sub_d(int R, bool start, const SubArgs &a, int blocks, hipStream_t s)
{
    auto go = [&](auto r_tag) {
        constexpr int RR = decltype(r_tag)::value;
        if (start)
            sub_start_launch<D, RR>(a, blocks, s);
        else
            sub_dp_launch<D, RR>(a, blocks, s);
    };
    switch (R) {
    case 1: go(std::integral_constant<int, 1>()); break;
    case 2: go(std::integral_constant<int, 2>()); break;
    case 4: go(std::integral_constant<int, 4>()); break;
    case 8: go(std::integral_constant<int, 8>()); break;
    default: go(std::integral_constant<int, 16>()); break;
    }
}

void launch_sub(int D, int R, bool start, const SubArgs &a, int blocks, hipStream_t s)
{
    switch (D) {
    case 1: sub_d<1>(R, start, a, blocks, s); break;
    case 2: sub_d<2>(R, start, a, blocks, s); break;
    case 3: sub_d<3>(R, start, a, blocks, s); break;
    case 4: sub_d<4>(R, start, a, blocks, s); break;
    case 5: sub_d<5>(R, start, a, blocks, s); break;
    case 6: sub_d<6>(R, start, a, blocks, s); break;
    case 7: sub_d<7>(R, start, a, blocks, s); break;
    default: sub_d<8>(R, start, a, blocks, s); break;
    }
}

void launch_sub_seed(int D, const SubArgs &a, int blocks, hipStream_t s)
{
    switch (D) {
#define TSK_SEED(DD)                                                                               \
    case DD:                                                                                       \
        hipLaunchKernelGGL(k_sub_rowmin<DD>, dim3(blocks), dim3(256), 0, s, a);                    \
        hipLaunchKernelGGL(k_sub_walk<DD>, dim3(blocks), dim3(256), 0, s, a, 0);                   \
        hipLaunchKernelGGL(k_sub_walk<DD>, dim3(blocks), dim3(256), 0, s, a, 1);                   \
        break;
        TSK_SEED(1)
        TSK_SEED(2)
        TSK_SEED(3)
        TSK_SEED(4)
        TSK_SEED(5)
        TSK_SEED(6)
        TSK_SEED(7)
        TSK_SEED(8)
#undef TSK_SEED
    default: break;
    }
}

int grid_of(int64_t n, int block, int cap)
{
    const int64_t g = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

void fill32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_of(n, 256, 4096)), dim3(256), 0, s, p, v, n);
}

void fill64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_of(n, 256, 4096)), dim3(256), 0, s, p, v, n);
}

// Buffers of one call, freed after the stream has drained.
struct SubBufs {
    hipStream_t s = nullptr;
    DevBuf<int64_t> qoff, soff, coff;
    DevBuf<uint32_t> pseed, pcnt, tau, pclb, plive;
    DevBuf<int64_t> live;
    DevBuf<int32_t> cj;
    DevBuf<unsigned long long> pbest, seedslots, resslots, work, ctr, nlive;
    DevBuf<float> clb;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    ~SubBufs()
    {
        (void)hipStreamSynchronize(s);
        qoff.release();
        soff.release();
        coff.release();
        pseed.release();
        pcnt.release();
        tau.release();
        pbest.release();
        seedslots.release();
        resslots.release();
        work.release();
        nlive.release();
        ctr.release();
        clb.release();
        pclb.release();
        plive.release();
        live.release();
        cj.release();
        for (auto &e : ev)
            if (e)
                (void)hipEventDestroy(e);
    }
};

int check_offsets(const int64_t *off, int64_t n, const char *what, int64_t max_len, int64_t *mx)
{
    if (!off)
        return set_err(TSK_ERR_INVALID_ARG, "%s offsets are NULL", what);
    if (n < 1)
        return set_err(TSK_ERR_INVALID_ARG, "%s count must be >= 1", what);
    if (n > INT32_MAX)
        return set_err(TSK_ERR_UNSUPPORTED, "%s count above 2^31-1", what);
    if (off[0] != 0)
        return set_err(TSK_ERR_INVALID_ARG, "%s offsets[0] must be 0", what);
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t L = off[i + 1] - off[i];
        if (L < 1)
            return set_err(TSK_ERR_INVALID_ARG, "%s %lld has length %lld (must be >= 1)", what,
                           (long long)i, (long long)L);
        if (L > max_len)
            return set_err(TSK_ERR_UNSUPPORTED, "%s %lld has length %lld > %lld", what,
                           (long long)i, (long long)L, (long long)max_len);
        m = std::max(m, L);
    }
    *mx = m;
    return TSK_OK;
}

} // namespace

extern "C" int tsk_subseq_query(const float *series_dev, const int64_t *s_offsets_host,
                                int64_t n_series, int32_t dim, const float *q_values_dev,
                                const int64_t *q_offsets_host, int64_t n_queries, int32_t k,
                                const tsk_subseq_opts *opts, int64_t *out_ids_dev,
                                float *out_dist_dev, int64_t *out_end_dev, int64_t *out_start_dev,
                                tsk_stats *stats_host, void *hip_stream)
{
    g_err.clear();
    // ---- validation, before any device work
    if (!series_dev || !q_values_dev)
        return set_err(TSK_ERR_INVALID_ARG, "series_dev / q_values_dev is NULL");
    if (dim < 1 || dim > TSK_SUB_MAX_DIM)
        return set_err(TSK_ERR_UNSUPPORTED, "dim %d outside [1, %d]", dim, TSK_SUB_MAX_DIM);
    if (k < 1)
        return set_err(TSK_ERR_INVALID_ARG, "k must be >= 1");
    if (k > TSK_MAX_K)
        return set_err(TSK_ERR_UNSUPPORTED, "k %d > %d", k, TSK_MAX_K);
    if (!out_ids_dev || !out_dist_dev || !out_end_dev)
        return set_err(TSK_ERR_INVALID_ARG, "output pointers are NULL");
    int64_t max_n = 0, max_m = 0;
    TSK_TRY(check_offsets(s_offsets_host, n_series, "series", INT32_MAX, &max_n));
    TSK_TRY(check_offsets(q_offsets_host, n_queries, "query", TSK_SUB_MAX_QLEN, &max_m));
    tsk_subseq_opts o;
    memset(&o, 0, sizeof(o));
    o.size = sizeof(o);
    o.seed = 1;
    if (opts) {
        if (opts->size != (int64_t)sizeof(tsk_subseq_opts))
            return set_err(TSK_ERR_INVALID_ARG, "opts->size %lld != sizeof(tsk_subseq_opts) %zu",
                           (long long)opts->size, sizeof(tsk_subseq_opts));
        o = *opts;
    }
    if (o.chunk_cols < 0 || o.waves_per_cu < 0 || o.waves_per_cu > 32 || (o.seed != 0 && o.seed != 1))
        return set_err(TSK_ERR_INVALID_ARG, "opts: chunk_cols >= 0, waves_per_cu in [0, 32], seed 0/1");
    int dev = -1, n_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    TSK_TRY(check_dev_ptr(series_dev, dev, "series_dev"));
    TSK_TRY(check_dev_ptr(q_values_dev, dev, "q_values_dev"));
    TSK_TRY(check_dev_ptr(out_ids_dev, dev, "out_ids_dev"));
    TSK_TRY(check_dev_ptr(out_dist_dev, dev, "out_dist_dev"));
    TSK_TRY(check_dev_ptr(out_end_dev, dev, "out_end_dev"));
    TSK_TRY(check_dev_ptr(out_start_dev, dev, "out_start_dev"));
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    n_cu = std::max(1, n_cu);
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t N = n_series;
    const int D = dim;
    int R = 1;
    while (64 * R < max_m)
        R *= 2;
    // queries per group: per-pair state of at most 2^25 pairs
    const int64_t G = std::max<int64_t>(1, std::min<int64_t>(n_queries, ((int64_t)1 << 25) / N));
    int64_t total_cols = 0;
    for (int64_t c = 0; c < N; ++c)
        total_cols += s_offsets_host[c + 1] - s_offsets_host[c];
    int64_t C = o.chunk_cols;
    if (C == 0) {
        // about 2^18 items per group (one thread each in the row-minimum,
        // walk and compaction passes), 64 to 4096 columns each
        C = (total_cols * G + ((int64_t)1 << 18) - 1) >> 18;
        C = std::min<int64_t>(std::max<int64_t>(((C + 63) / 64) * 64, 64), 4096);
    }
    C = std::min<int64_t>(C, INT32_MAX);
    std::vector<int64_t> coff(N + 1, 0);
    for (int64_t c = 0; c < N; ++c)
        coff[c + 1] = coff[c] + (s_offsets_host[c + 1] - s_offsets_host[c] + C - 1) / C;
    const int64_t chunks = coff[N];

    SubBufs b;
    b.s = s;
    TSK_TRY(b.qoff.ensure(G + 1));
    TSK_TRY(b.soff.ensure(N + 1));
    TSK_TRY(b.coff.ensure(N + 1));
    TSK_TRY(b.pseed.ensure(G * N));
    TSK_TRY(b.pcnt.ensure(G * N));
    TSK_TRY(b.pbest.ensure(G * N));
    TSK_TRY(b.tau.ensure(G));
    TSK_TRY(b.seedslots.ensure(G * k));
    TSK_TRY(b.resslots.ensure(G * k));
    TSK_TRY(b.work.ensure(1));
    TSK_TRY(b.ctr.ensure(CTR_WORDS));
    TSK_TRY(b.clb.ensure(G * chunks));
    TSK_TRY(b.cj.ensure(G * chunks));
    TSK_TRY(b.pclb.ensure(G * N));
    TSK_TRY(b.plive.ensure(G * N));
    TSK_TRY(b.live.ensure(G * chunks));
    TSK_TRY(b.nlive.ensure(1));
    for (auto &e : b.ev)
        HIP_TRY(hipEventCreate(&e));
    HIP_TRY(hipMemcpyAsync(b.soff.p, s_offsets_host, (N + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b.coff.p, coff.data(), (N + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    fill64(b.ctr.p, 0ull, CTR_WORDS, s);
    const int waves = o.waves_per_cu ? o.waves_per_cu : 16;
    const int dp_blocks = std::max(1, n_cu * waves / 4);
    float t_seed = 0, t_dp = 0, t_fin = 0, t_all = 0;
    std::vector<int64_t> hq;
    for (int64_t q0 = 0; q0 < n_queries; q0 += G) {
        const int64_t g = std::min<int64_t>(G, n_queries - q0);
        hq.assign(q_offsets_host + q0, q_offsets_host + q0 + g + 1);
        for (auto &v : hq)
            v -= q_offsets_host[q0];
        HIP_TRY(hipMemcpyAsync(b.qoff.p, hq.data(), (g + 1) * sizeof(int64_t),
                               hipMemcpyHostToDevice, s));
        SubArgs a;
        memset(&a, 0, sizeof(a));
        a.qv = q_values_dev + q_offsets_host[q0] * D;
        a.qoff = b.qoff.p;
        a.nq = (int)g;
        a.ser = series_dev;
        a.soff = b.soff.p;
        a.N = N;
        a.coff = b.coff.p;
        a.chunks = chunks;
        a.C = (int)C;
        a.k = k;
        a.pseed = b.pseed.p;
        a.pbest = b.pbest.p;
        a.pcnt = b.pcnt.p;
        a.clb = b.clb.p;
        a.cj = b.cj.p;
        a.pclb = b.pclb.p;
        a.plive = b.plive.p;
        a.live = b.live.p;
        a.nlive = b.nlive.p;
        a.seedslots = b.seedslots.p;
        a.resslots = b.resslots.p;
        a.tau = b.tau.p;
        a.work = b.work.p;
        a.ctr = b.ctr.p;
        a.out_ids = out_ids_dev + q0 * k;
        a.out_dist = out_dist_dev + q0 * k;
        a.out_end = out_end_dev + q0 * k;
        a.out_start = out_start_dev ? out_start_dev + q0 * k : nullptr;
        HIP_TRY(hipEventRecord(b.ev[0], s));
        fill32(b.pseed.p, TSK_INF_BITS, g * N, s);
        fill32(b.pclb.p, TSK_INF_BITS, g * N, s);
        fill32(b.plive.p, 0u, g * N, s);
        fill64(b.nlive.p, 0ull, 1, s);
        fill32(b.pcnt.p, 0u, g * N, s);
        fill64(b.pbest.p, TSK_KEY_EMPTY, g * N, s);
        fill32(b.tau.p, TSK_INF_BITS, g, s);
        fill64(b.seedslots.p, TSK_KEY_EMPTY, g * k, s);
        fill64(b.resslots.p, TSK_KEY_EMPTY, g * k, s);
        fill64(b.work.p, 0ull, 1, s);
        if (o.seed) {
            launch_sub_seed(D, a, grid_of(g * chunks, 256, 1 << 16), s);
            hipLaunchKernelGGL(k_sub_seed_topk, dim3(grid_of(g * N, 256, 1 << 16)), dim3(256), 0,
                               s, a);
        } else {
            fill32((uint32_t *)b.clb.p, 0u, g * chunks, s); // row-0 minima unknown: skip nothing
        }
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_sub_compact, dim3(grid_of(g * chunks, 256, 1 << 16)), dim3(256), 0,
                           s, a);
        HIP_TRY(hipEventRecord(b.ev[1], s));
        launch_sub(D, R, false, a, dp_blocks, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(b.ev[2], s));
        hipLaunchKernelGGL(k_sub_finalize, dim3(grid_of(g * k, 256, 1 << 16)), dim3(256), 0, s, a);
        if (out_start_dev)
            launch_sub(D, R, true, a, grid_of(g * k, 4, 1 << 16), s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(b.ev[3], s));
        HIP_TRY(hipEventSynchronize(b.ev[3]));
        float x = 0;
        HIP_TRY(hipEventElapsedTime(&x, b.ev[0], b.ev[1]));
        t_seed += x;
        HIP_TRY(hipEventElapsedTime(&x, b.ev[1], b.ev[2]));
        t_dp += x;
        HIP_TRY(hipEventElapsedTime(&x, b.ev[2], b.ev[3]));
        t_fin += x;
        HIP_TRY(hipEventElapsedTime(&x, b.ev[0], b.ev[3]));
        t_all += x;
    }
    if (stats_host) {
        unsigned long long words[CTR_WORDS], c[C_NUM];
        HIP_TRY(hipMemcpyAsync(words, b.ctr.p, sizeof(words), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        ctr_sum(words, c);
        memset(stats_host, 0, sizeof(*stats_host));
        stats_host->pairs = n_queries * N;
        stats_host->seed_pairs = (int64_t)c[C_SEED_PAIRS];
        stats_host->bound_pruned = (int64_t)c[C_BOUND_PRUNED];
        stats_host->dp_started = (int64_t)c[C_DP_STARTED];
        stats_host->dp_completed = (int64_t)c[C_DP_COMPLETED];
        stats_host->dp_abandoned = (int64_t)c[C_DP_ABANDONED];
        stats_host->dp_cells = (int64_t)c[C_DP_CELLS];
        stats_host->bound_steps = (int64_t)c[C_BOUND_STEPS];
        stats_host->dp_valid_cells = (int64_t)c[C_VALID_CELLS];
        stats_host->calls = 1;
        stats_host->ms_total = t_all;
        stats_host->ms_seed = t_seed;
        stats_host->ms_dp = t_dp;
        stats_host->ms_final = t_fin;
    }
    HIP_TRY(hipStreamSynchronize(s));
    return TSK_OK;
}
