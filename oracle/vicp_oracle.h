/* vicp_oracle.h -- declarations of the CPU oracle (test infrastructure only;
 * see vicp_oracle.c).  Arrays are structure-of-arrays float32 coordinates;
 * grids are described by origin[3], inv = 1/voxel, dims[3] and V. */
#ifndef VICP_ORACLE_H
#define VICP_ORACLE_H
#include <stdint.h>

#define VICPO_OK 0
#define VICPO_ERR_ARG (-1)
#define VICPO_ERR_TOO_LARGE (-2)
#define VICPO_ERR_OOM (-3)
#define VICPO_ERR_NONFINITE (-4)
#define VICPO_ERR_INTERNAL (-5)

int vicpo_set_threads(int32_t k);
int vicpo_grid_spec(const float* qx, const float* qy, const float* qz, int64_t n,
                    float voxel, int32_t rings, float origin[3], float* inv,
                    int32_t dims[3], int64_t* V);
int vicpo_voxel_ids(const float* x, const float* y, const float* z, int64_t k,
                    const float origin[3], float inv, const int32_t dims[3], int64_t* out);
int vicpo_build(const float* qx, const float* qy, const float* qz, int64_t n,
                const float origin[3], float inv, const int32_t dims[3], int64_t V,
                uint32_t* hist, uint32_t* off, uint32_t* vm);
int vicpo_dilate(const int32_t dims[3], int64_t V, const uint32_t* hist,
                 const uint32_t* off, int32_t rings, uint32_t* vm, uint32_t* roots_out);
int vicpo_nns(const float* qx, const float* qy, const float* qz, int64_t n,
              const float origin[3], float inv, const int32_t dims[3],
              const uint32_t* off, const uint32_t* vm,
              const float* px, const float* py, const float* pz, int64_t m,
              const float Rt[12], int32_t* nn_idx, float* nn_d2, int64_t* n_fallback,
              int64_t* cand_total, int64_t* dilated_total);
int vicpo_nns_cap(const float* qx, const float* qy, const float* qz, int64_t n,
                  const float origin[3], float inv, const int32_t dims[3],
                  const uint32_t* off, const uint32_t* vm,
                  const float* px, const float* py, const float* pz, int64_t m,
                  const float Rt[12], int64_t capacity, int32_t* nn_idx, float* nn_d2,
                  int64_t* n_fallback, int64_t* cand_total, int64_t* dilated_total);
int vicpo_solve(const float* px, const float* py, const float* pz,
                const float* qx, const float* qy, const float* qz,
                const int32_t* idx, int64_t m, const double Rt_prev[12],
                double Rt_out[12], double sv_out[3], int32_t* degenerate);
int vicpo_register(const float* qx, const float* qy, const float* qz, int64_t n,
                   const float* px, const float* py, const float* pz, int64_t m,
                   float voxel, int32_t rings, int32_t max_iter, double rmse_eps,
                   int32_t early_stop, double Rt_io[12], double* rmse_hist,
                   int64_t* fb_hist, int32_t* iters_done, int32_t* degenerate_hist,
                   int32_t* nn_idx, float* nn_d2);
int vicpo_register_spec(const float* qx, const float* qy, const float* qz, int64_t n,
                        const float* px, const float* py, const float* pz, int64_t m,
                        const float origin[3], float inv, const int32_t dims[3], int64_t V,
                        int32_t rings, int32_t max_iter, double rmse_eps,
                        int32_t early_stop, double Rt_io[12], double* rmse_hist,
                        int64_t* fb_hist, int32_t* iters_done, int32_t* degenerate_hist,
                        int32_t* nn_idx, float* nn_d2);
int vicpo_register_cap(const float* qx, const float* qy, const float* qz, int64_t n,
                       const float* px, const float* py, const float* pz, int64_t m,
                       const float origin[3], float inv, const int32_t dims[3], int64_t V,
                       int32_t rings, int64_t capacity, int32_t max_iter, double rmse_eps,
                       int32_t early_stop, double Rt_io[12], double* rmse_hist,
                       int64_t* fb_hist, int32_t* iters_done, int32_t* degenerate_hist,
                       int32_t* nn_idx, float* nn_d2);
void vicpo_se3_exp(const double xi[6], double R[9], double t[3], double Jl6[36]);
double vicpo_p2p_loss_fixed(const float* qx, const float* qy, const float* qz,
                            const double* px, const double* py, const double* pz, int64_t m,
                            const int32_t* idx, const double xi[6]);
int vicpo_p2p(const float* qx, const float* qy, const float* qz, int64_t n,
              const float origin[3], float inv, const int32_t dims[3],
              const uint32_t* off, const uint32_t* vm,
              const float* px, const float* py, const float* pz, int64_t m,
              const double xi[6], double* loss, double* dpx, double* dpy, double* dpz,
              double dxi[6], int32_t* nn_idx);
#endif
