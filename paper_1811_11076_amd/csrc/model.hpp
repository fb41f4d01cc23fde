// The encoder object behind tsk_model and the pieces of it that the k-NN
// query uses for TSK_ORDER_LEARNED.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "runtime.hpp"

struct tsk_model {
    int device = 0;
    int dim = 0, points = 32, d_in = 0, hidden = 256, embed = 64;
    int64_t n_params = 0;
    int64_t off[7] = {0}; // W1, b1, W2, b2, W3, b3, end (floats)
    tsk::DevBuf<float> params, grads, m, v;
    int64_t step = 0;
    uint64_t uid = 0;     // unique per model object
    uint64_t version = 1; // bumped whenever the parameters change
    // scratch of the forward / backward passes
    tsk::DevBuf<float> x, a1, a2, e, de, g2, g1, loss, pool, y;
    tsk::DevBuf<int64_t> off_dev;
    tsk::DevBuf<int32_t> ia, ib;
    std::mutex mu;
};

namespace tsk {

// Rows of series embedded per pass of model_embed_dev.
constexpr int64_t EMBED_CHUNK = 65536;

// Sizes the encoder's scratch for passes of `rows` series (allocates only if
// it grows; a captured embedding pass needs it sized beforehand).
int model_reserve_rows(tsk_model *mdl, int64_t rows);

// Embeddings of n series (AoS values, device offsets) into out [n][embed],
// in chunks of rows; asynchronous on s.
int model_embed_dev(tsk_model *mdl, const float *vals, const int64_t *off_dev, int64_t n,
                    float *out, hipStream_t s);

// S[q][c] = squared distance of query embedding q and candidate embedding c.
void launch_embed_score(const float *Eq, int nq, const float *Ec, int64_t N, int width, float *S,
                        hipStream_t s);

// order[q][0..N) = candidates of query q by ascending S[q][.] (bucketed).
void launch_bucket_order(const float *S, int nq, int64_t N, int32_t *order, hipStream_t s);

} // namespace tsk
