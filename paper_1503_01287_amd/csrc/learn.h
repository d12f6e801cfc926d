// Learned per-level damping of the Jacobi smoother: row statistics of A_l
// (the network's input features) and the network 8 -> 32 -> 32 -> 1 with
// its training kernels (forward, backward, Adam). All of it is tiny and
// latency bound; it runs once per setup (inference) or offline (training).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace amgp2 {

constexpr int MLP_NF = 8, MLP_NH = 32;
// flat parameter layout: W1 (32x8), b1, W2 (32x32), b2, W3 (32), b3
constexpr int MLP_OW1 = 0, MLP_OB1 = MLP_OW1 + MLP_NH * MLP_NF, MLP_OW2 = MLP_OB1 + MLP_NH,
              MLP_OB2 = MLP_OW2 + MLP_NH * MLP_NH, MLP_OW3 = MLP_OB2 + MLP_NH, MLP_OB3 = MLP_OW3 + MLP_NH,
              MLP_NP = MLP_OB3 + 1;
constexpr float MLP_OMEGA_MIN = 0.2f, MLP_OMEGA_SPAN = 1.0f;

// The eight features of a level (see amg_level_features in the public header).
// mode 3: 3x3 blocks (planes); mode 1: scalar operator applied per component.
void row_features(int mode, int n, const int *rowptr, const int *col, const double *val, int64_t nnz, int level,
                  double *features_host, hipStream_t s);

// The same features written to f_dev (8 device doubles), stream-ordered,
// with every intermediate in scratch_dev (features_scratch_address()): no
// allocation, no host synchronisation. Levels of more than
// features_noalloc_max_rows() scalar rows are rejected (AMG_EINVAL).
void row_features_noalloc(int mode, int n, const int *rowptr, const int *col, const double *val, int64_t nnz,
                          int level, double *scratch_dev, double *f_dev, hipStream_t s);
int features_noalloc_max_rows();
double *features_scratch_address();

struct MlpWork {
    int cap = 0;
    DevBuf<float> X, y, H1, H2, S, om, D1, D2, D3, err2;
    void reserve(int n);
};

// omega = 0.2 + sigmoid(z) for every sample (device pointers)
void mlp_forward(const float *theta, const float *X, int n, MlpWork &w, hipStream_t s);
// gradient of the mean squared error to y (device) after mlp_forward; loss -> *loss_dev
void mlp_backward(const float *theta, int n, MlpWork &w, float *grad, float *loss_dev, hipStream_t s);
// one Adam step with bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t
void mlp_adam(float *theta, const float *grad, float *m, float *v, float lr, float beta1, float beta2, float c1,
              float c2, float eps, hipStream_t s);

}  // namespace amgp2

// A network and its Adam state (the handle behind amg_mlp_handle).
struct amg_mlp {
    hipStream_t stream = nullptr;
    amgp2::DevBuf<float> theta, m, v, grad, loss;
    int t = 0;  // Adam steps taken
    amgp2::MlpWork w;
};

