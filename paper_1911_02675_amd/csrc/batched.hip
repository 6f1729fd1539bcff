// Batched form: many independent problems in one persistent launch.
#include "internal.h"

extern "C" lsq_status lsq_pcg_solve_batched(lsq_ctx* ctx, int32_t count, const lsq_problem* probs,
                                            const lsq_sketch_desc* descs, const lsq_pcg_opts* opts,
                                            double* const* xs, lsq_info* infos) {
  (void)ctx; (void)count; (void)probs; (void)descs; (void)opts; (void)xs; (void)infos;
  return LSQ_ERR_UNSUPPORTED;
}
