// Entry points of the batch and learned-preconditioner layers that are not
// built yet: they report MXSEM_ENOTSUP.
#include "runtime.hpp"

extern "C" {
int mxsem_fcg_solve_impl(mxsem_mesh*, const mxsem_solve_opts*, const double*, double*,
                         mxsem_solve_stats*) {
  mx::set_error("flexible CG is not available in this build");
  return MXSEM_ENOTSUP;
}
int mxsem_nn_create(mxsem_mesh*, const mxsem_nn_desc*, mxsem_nn**) { return MXSEM_ENOTSUP; }
int mxsem_nn_destroy(mxsem_nn*) { return MXSEM_OK; }
int mxsem_nn_set_params(mxsem_nn*, const float*, const float*) { return MXSEM_ENOTSUP; }
int mxsem_nn_get_params(mxsem_nn*, float*, float*) { return MXSEM_ENOTSUP; }
int mxsem_nn_forward(mxsem_nn*, const float*, float*) { return MXSEM_ENOTSUP; }
int mxsem_nn_loss_grad(mxsem_nn*, const float*, const float*, int, double*, float*) { return MXSEM_ENOTSUP; }
int mxsem_nn_adam_step(mxsem_nn*, const mxsem_adam*) { return MXSEM_ENOTSUP; }
int mxsem_mesh_attach_nn(mxsem_mesh*, mxsem_nn*) { return MXSEM_ENOTSUP; }
}
