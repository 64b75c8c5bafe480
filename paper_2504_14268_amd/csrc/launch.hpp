// launch.hpp -- host-side launchers of the kernels in kernels.hip.
#pragma once
#include "kernels.hpp"

namespace mpcg {
void launch_start(const KArgs &a, hipStream_t s);
void launch_slot(const KArgs &a, hipStream_t s);
// With events e0/e1 the launch records the kernel's own start and stop times.
void launch_ka(const KArgs &a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_kb(const KArgs &a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_kx(const KArgs &a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_step_x(const KArgs &a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_step_b(const KArgs &a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_finish(const KArgs &a, hipStream_t s);
void launch_batched(const BatchSys *sys, const int32_t *order, int nsys, int32_t *queue, int grid,
                    hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_lock_slot(const BatchSys *sys, const SysBlk *tka, int nka, const SysBlk *tvb, int nvb,
                      const int32_t *act, int nact, int slow, hipStream_t s);
void launch_lock_start(const BatchSys *sys, const SysBlk *tvb, int nvb, hipStream_t s);
void launch_lock_finish(const BatchSys *sys, const SysBlk *tka, int nka, const SysBlk *tvb, int nvb,
                        const int32_t *act, int nact, int slow, hipStream_t s);
void launch_lock_modes(const BatchSys *sys, const int32_t *act, int nact, int32_t *modes, hipStream_t s);
void launch_pack16(int np, const uint16_t *v, const int16_t *dc, uint32_t *out, hipStream_t s);
void launch_dcol(int n, const int *rp, const int *ci, int16_t *dc, int *bad, hipStream_t s);
void launch_shadows(int n, const int *rp, const int *ci, const double *v, float *v32, uint16_t *vbf,
                    uint16_t *vh, uint8_t *v8, float *vtf, int8_t *rexp, float *minv, hipStream_t s);
void launch_op_spmv(const Mat &A, int fs, int tier, const void *p, void *q, hipStream_t s);
void launch_op_residual(const Mat &A, const double *b, const double *x, double *r, hipStream_t s);
void launch_op_dot(int n, int fd, int tier, const void *u, const void *v, double *part, int P2, double *out,
                   hipStream_t s);
// launch_op_dot with its partials in the library's static device array (at
// most kNoAllocPartials blocks of kVecBlock elements); no allocation.
hipError_t launch_op_dot_noalloc(int n, int fd, int tier, const void *u, const void *v, double *out,
                                 hipStream_t s);
void launch_op_axpy(int n, int fa, double alpha, const void *u, void *y, hipStream_t s);
// Flat gather of p over the CSR column stream (measurement of the random-access floor).
void launch_gather_floor(const Mat &A, const float *p, float *sink, hipStream_t s);
// One slot of the single-reduction CG (KS1 then KS2).
void launch_sr_slot(const SrArgs &a, hipStream_t s);
void launch_policy_decide(const PolicyDev *P, int m, const int64_t *k, const double *rho, const int32_t *stag,
                          const float *feat, int32_t *state, int32_t *action, hipStream_t s);
}  // namespace mpcg
