// Host driver of the SPPM iteration (implemented in sppm.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "pm.h"

namespace pm {

int sppm_validate(const pm_scene_desc *d, const pm_sppm_params *p);
int sppm_create(const pm_scene_desc *d, const pm_sppm_params *p, hipStream_t st, pm_sppm **out);
int sppm_destroy(pm_sppm *s);
int sppm_iterate(pm_sppm *s, int32_t n_iter, hipStream_t st);
int sppm_resolve(pm_sppm *s, float *image, hipStream_t st);
int sppm_status(pm_sppm *s, hipStream_t st);
int sppm_views(pm_sppm *s, pm_sppm_views *v);
int sppm_save(pm_sppm *s, void *buf, uint64_t *size, hipStream_t st);
int sppm_load(pm_sppm *s, const void *buf, uint64_t size, hipStream_t st);
int sppm_get_stats(pm_sppm *s, pm_sppm_stats *out, int32_t reset, hipStream_t st);
int sppm_adjoint(pm_sppm *s, const float *g, const int32_t *pmat, int32_t n_par, double *grad, hipStream_t st);

int batch_create(const pm_scene_desc *const *descs, const pm_sppm_params *const *params, int32_t n,
                 const pm_batch_opts *opts, hipStream_t st, pm_batch **out);
int batch_destroy(pm_batch *b);
int batch_iterate(pm_batch *b, int32_t n, hipStream_t st);
int batch_resolve(pm_batch *b, float *const *images, hipStream_t st);
int batch_status(pm_batch *b, hipStream_t st);
int batch_info(const pm_batch *b, pm_batch_info *info);
int batch_views(pm_batch *b, int32_t scene, pm_sppm_views *v);

}  // namespace pm
