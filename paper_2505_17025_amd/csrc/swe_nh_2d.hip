// swe_nh_2d.hip -- 2D path (placeholder until the 2D kernels land)
#include "swe_nh_2d.h"

namespace swenh {
void plan2d(const swe_nh_config*, char*, size_t*, Ctx2D*) {}
int init2d(const swe_nh_config*, Ctx2D*, const K1D&, hipStream_t) { return SWE_NH_EINVAL; }
void enqueue_step2d(const swe_nh_config*, Ctx2D*, hipStream_t, double*, double*, double*, double*,
                    double*, uint8_t*) {}
void launch_pred2d_stage(const swe_nh_config*, Ctx2D*, hipStream_t, const double*, const double*,
                         const double*, const double*, const double*, const double*, double*,
                         double*, double*, double*) {}
void launch_mask2d_stage(const swe_nh_config*, Ctx2D*, hipStream_t, const double*, const double*,
                         const double*, const double*, const double*, int, uint8_t*) {}
void solve_pressure2d(const swe_nh_config*, Ctx2D*, hipStream_t, const double*, const double*,
                      const double*, const double*, const uint8_t*, const double*, const double*,
                      double*) {}
void correct2d(const swe_nh_config*, Ctx2D*, hipStream_t, const double*, const double*,
               const double*, const double*, const uint8_t*, const double*, const double*,
               const double*, double*, double*, double*) {}
void time_stage2d(const swe_nh_config*, Ctx2D*, hipStream_t, int, double*, double*, double*,
                  double*, double*) {}
}  // namespace swenh
