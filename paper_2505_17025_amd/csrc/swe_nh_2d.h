// swe_nh_2d.h -- 2D path (structured [ny][nx] grid): context and entry points
// used by the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swe_nh.h"
#include "swe_nh_kernels.h"

namespace swenh {

struct Ctx2D {
  int* n_act = nullptr;
  int* iters = nullptr;
  double* rel = nullptr;
};

void plan2d(const swe_nh_config* c, char* base, size_t* off, Ctx2D* x);
int init2d(const swe_nh_config* c, Ctx2D* x, const K1D& k1, hipStream_t s);
void enqueue_step2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, double* h, double* hu,
                    double* hv, double* hw, double* p, uint8_t* mask);
void launch_pred2d_stage(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* h,
                         const double* hu, const double* hv, const double* hw, const double* t_in,
                         const double* dt_in, double* ht, double* mt, double* nt, double* kt);
void launch_mask2d_stage(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* ht,
                         const double* mt, const double* nt, const double* kt,
                         const double* t_in, int mode, uint8_t* mask);
void solve_pressure2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* ht,
                      const double* mt, const double* nt, const double* kt, const uint8_t* mask,
                      const double* t_in, const double* dt_in, double* p);
void correct2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* ht,
               const double* mt, const double* nt, const double* kt, const uint8_t* mask,
               const double* p, const double* t_in, const double* dt_in, double* m_out,
               double* n_out, double* k_out);

void time_stage2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, int stage, double* h,
                  double* hu, double* hv, double* hw, double* p);

}  // namespace swenh
