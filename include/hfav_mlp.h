/*
 * hfav_mlp.h - the learned tile-configuration cost model.
 *
 * A multilayer perceptron (three ReLU hidden layers of width H, one linear
 * output) maps the features of a chain and of a candidate kernel
 * configuration to the predicted log time per cell.  The GPU entry points
 * train it (FP32 forward, backward and Adam kernels); the host entry points
 * give the candidate set and the feature vector (the same code serves the
 * autotuner and the planner) and install trained weights, after which
 * hfav_plan with config_source = HFAV_CONFIG_MODEL picks the candidate with
 * the smallest predicted time.
 *
 * The paper tunes nothing automatically; this extension is the project's
 * own (the network, its 24 features and the candidate set), trained with
 * Adam (Kingma and Ba, 2015) on mean squared error.
 *
 * Parameters are one flat float array: W1 (H,d) b1 (H) W2 (H,H) b2 (H)
 * W3 (H,H) b3 (H) W4 (1,H) b4 (1), row-major W[out][in].
 * Device entry points take DEVICE pointers and enqueue on `stream`; they
 * return 0, or 1 for a bad argument, 8 for a HIP error.
 */
#ifndef HFAV_MLP_H
#define HFAV_MLP_H

#include <stddef.h>

#include "hfav.h"

#ifdef __cplusplus
extern "C" {
#endif

#define HFAV_COST_FEATURES 24
#define HFAV_MAX_CANDIDATES 64

/* number of parameters of the network */
size_t hfav_mlp_nparams(int d, int H);
/* device workspace the training and inference calls need for n samples */
size_t hfav_mlp_workspace_bytes(int n, int d, int H);

/* y (n) = network(X (n,d)) */
int hfav_mlp_forward(const float *X, int n, int d, int H, const float *params, float *y, void *workspace,
                     void *stream);
/* loss = mean (y - t)^2 (device scalar, nullable) and its gradient G (same
 * layout as params) by backpropagation */
int hfav_mlp_loss_grad(const float *X, const float *t, int n, int d, int H, const float *params, float *grads,
                       float *loss, void *workspace, void *stream);
/* one Adam step (bias-corrected, step >= 1) on params with moments m, v */
int hfav_mlp_adam(float *params, const float *grads, float *m, float *v, int np, float lr, float b1, float b2,
                  float eps, int step, void *stream);

/* Candidate configurations of a chain of linear star stages at a grid size
 * (host, no GPU): every group depth, tile shape and segment length whose
 * fused groups fit in LDS.  Returns the count (<= max), or -1 if the chain
 * is not such a chain. */
int hfav_star_candidates(hfav_chain *chain, const int dims[3], hfav_config *out, int max);

/* Feature vector (HFAV_COST_FEATURES floats) of a chain, grid size and
 * configuration (host).  Returns 0, or an hfav_status on error. */
int hfav_costmodel_features(hfav_chain *chain, const int dims[3], const hfav_config *cfg, float *out);

/* Install trained weights (host arrays, copied): H hidden width, feature
 * normalisation mean/std (HFAV_COST_FEATURES each).  params = NULL removes
 * the model. */
int hfav_costmodel_set(const float *params, int H, const float *mean, const float *std);

/* Predicted log time per cell of a configuration with the installed model. */
int hfav_costmodel_predict(hfav_chain *chain, const int dims[3], const hfav_config *cfg, float *out);

#ifdef __cplusplus
}
#endif
#endif /* HFAV_MLP_H */
