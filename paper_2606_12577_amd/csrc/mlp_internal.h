// Internal declarations of the block-smoother network (learned setup).
#pragma once

#include "cs_internal.h"
#include "../../include/cascade_learned.h"

namespace cs {

struct Mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int n_in = 0, width = 0, n_out = 0;
    int64_t np = 0;                       // parameter count
    int64_t off[7] = {0};                 // W1, b1, W2, b2, W3, b3, end
    DBuf<float> p, g, m, v;               // parameters, gradient, Adam moments
    DBuf<float> mean, std;                // output scaling
    int64_t step = 0;                     // Adam steps taken
    // activations of one batch (capacity rows)
    int64_t cap = 0;
    DBuf<float> z1, h1, z2, h2, y, dy, d2, d1;
    DBuf<double> part, acc;               // loss partial sums
    DBuf<float> kpart;                    // split-k partial products
    double *h_acc = nullptr;              // pinned readback
    size_t h_acc_cap = 0;
};

// Y = prediction in target units for n rows of X (on stream s)
void mlp_predict(Mlp &m, hipStream_t s, const float *X, int64_t n, float *Y);

}  // namespace cs

struct cs_mlp_s {
    cs::Mlp m;
};
