#include "internal.hpp"
extern "C" {
int spgemm_backward(spg_plan, const spg_csr *, const spg_csr *, const spg_csr *, spg_dtype, void *,
                    void *, void *) { return SPG_ERR_UNSUPPORTED; }
int spgemm_mcl_workspace_size(int32_t, int32_t, size_t *) { return SPG_ERR_UNSUPPORTED; }
int spgemm_mcl_iteration(spg_plan, const spg_csr *, int32_t, float, int32_t, int32_t *, int32_t *,
                         float *, int64_t, int64_t *, void *, size_t, void *) {
  return SPG_ERR_UNSUPPORTED;
}
}
