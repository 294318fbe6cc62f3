// Learned warm start of the GenEO eigensolver (see model.hip).
#pragma once

#include "precond.h"

struct geneo_model {
  int32_t C = 12, hidden = 256, k = 20;
  int32_t in_dim = 0, rows = 0;
  int64_t R = 0;                          // rows * k outputs
  uint64_t seed = 0;
  std::vector<int32_t> edge_id;           // [7 * (C+1)^3] canvas edge (direction, low node) -> row, or -1
  // parameters: 0 W1 [hidden x in], 1 b1, 2 W2 [hidden x hidden], 3 b2, 4 W3 [R x hidden], 5 b3
  int64_t psize[6] = {0, 0, 0, 0, 0, 0};
  geneo::DevBuf<float> p32[6], m1[6], m2[6];  // FP32 master values, Adam moments
  geneo::DevBuf<uint16_t> pbf[6];             // BF16 copies used by the kernels (weights; biases stay FP32)
  int64_t adam_t = 0;
  // collected samples (host): features, targets over the canvas, row masks
  std::vector<float> feat, targ;
  std::vector<uint8_t> mask;
  std::vector<uint8_t> holdout;
};

namespace geneo {

// Fill the first min(k_model, nev) columns of the eigensolver's start block
// X (batch layout: subdomain j at voff[j] * kb, column q at + q * n_pad_j,
// already holding a random block) from the model, adding 1e-4 of the
// random block so that the columns stay independent.  Returns the number
// of subdomains that received a learned start.
int model_warm_start(geneo_ctx* ctx, const geneo_model* m, const geneo_precond* pc, int kb, int nev, double* X);

void model_init(geneo_model* m, const geneo_model_opts* o, hipStream_t st);
void model_collect(geneo_ctx* ctx, geneo_model* m, const geneo_system* s, const geneo_decomp* dec,
                   const geneo_precond* pc, int holdout);
void model_train(geneo_ctx* ctx, geneo_model* m, const geneo_train_opts* o, geneo_train_info* info);
void model_predict(geneo_ctx* ctx, const geneo_model* m, int B, const float* X, float* Y);
double model_loss_grad(geneo_ctx* ctx, const geneo_model* m, int B, const float* X, const float* V,
                       const uint8_t* mask, float* grad);
int64_t model_n_params(const geneo_model* m);
void model_get_params(const geneo_model* m, float* out);
// round_masters: store the BF16-rounded values as the FP32 masters too
void model_set_params(geneo_ctx* ctx, geneo_model* m, const float* in, bool round_masters);
void model_save(const geneo_model* m, const char* path);
void model_load(geneo_ctx* ctx, geneo_model* m, const char* path);

}  // namespace geneo
