// Learned boundary force (MLP 10-64-64-3): placeholder until the MFMA kernels land.
#include "common.h"

void mlp_step_forcing(iblbm_ctx*) {}

extern "C" {
iblbm_status iblbm_set_mlp(iblbm_ctx* c, const float*, const float*) {
  if (c) c->err = "learned forcing is not available in this build";
  return IBLBM_E_ARG;
}
iblbm_status iblbm_capture_samples(iblbm_ctx* c, float*, float*) {
  if (c) c->err = "learned forcing is not available in this build";
  return IBLBM_E_ARG;
}
iblbm_status iblbm_nn_train(const float*, const float*, int64_t, float*, const iblbm_train_opts*, float*) {
  return IBLBM_E_ARG;
}
iblbm_status iblbm_nn_grad(const float*, const float*, int64_t, const float*, float*, float*) {
  return IBLBM_E_ARG;
}
iblbm_status iblbm_nn_forward(const float*, int64_t, const float*, float*) { return IBLBM_E_ARG; }
}
