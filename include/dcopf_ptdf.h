/*
 * dcopf_ptdf.h - the PTDF matrix of a network, built on the GPU (Section 2:
 * the DCOPF line constraints in PTDF form use H_a, which maps bus injections,
 * withdrawn at the slack bus, to line flows).
 *
 * With E the line-bus incidence matrix (+1 at a line's from bus, -1 at its
 * to bus), E_r its columns without the slack bus and Omega = diag(b) the
 * series susceptances,
 *
 *     H_a[:, kept buses] = Omega E_r B_r^{-1},  B_r = E_r^T Omega E_r,
 *     H_a[:, slack] = 0.
 *
 * Computed in FP64 with dense factorisations on the matrix cores, blocks of
 * 64: B_r = L L^T (right-looking blocked Cholesky), W = L^{-1} (blocked
 * forward substitution on the identity), B_r^{-1} = W^T W, and row l of H_a
 * is b_l (B_r^{-1}[f_l] - B_r^{-1}[t_l]) on the kept buses.  About
 * (n_bus - 1)^3 flops.  Device workspace: two (n_bus - 1)^2 matrices of
 * doubles (rounded up to multiples of 64), allocated and freed by the call.
 * B_r is assembled row by row from the lines incident to each bus, in line
 * order, so the result does not depend on scheduling.
 */
#ifndef DCOPF_PTDF_H
#define DCOPF_PTDF_H

#include <stdint.h>

#include "dcopf_dual.h"

#ifdef __cplusplus
extern "C" {
#endif

/* fbus, tbus, b: HOST arrays [n_line] (bus indices in [0, n_bus), line
 * susceptances).  H: DEVICE buffer of n_line * n_bus doubles, row-major,
 * owned by the caller, written on hip_stream (NULL: the default stream);
 * the call synchronises that stream before returning.  Errors:
 * DCOPF_E_INVALID for n_bus < 2, n_line < 1, an index out of range, a line
 * whose two ends coincide, a susceptance that is not finite and positive,
 * a NULL pointer, or a network that is not connected (a pivot of the
 * Cholesky factorisation that is not positive; H is then unspecified);
 * DCOPF_E_NOMEM; DCOPF_E_HIP.                                             */
dcopf_status dcopf_ptdf(int32_t n_bus, int32_t n_line, const int32_t *fbus,
                        const int32_t *tbus, const double *b, int32_t slack,
                        void *hip_stream, double *H);

/* The same build without any device allocation, for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc / hipFree).  Arguments, result and errors as dcopf_ptdf; the
 * kernels and their order are the same, so H is bitwise equal to what
 * dcopf_ptdf writes.  The workspace is a fixed device array inside the
 * library (about 65 MiB, allocated with the code object on each device the
 * library runs on and held until the process ends), so the network must
 * have at most DCOPF_PTDF_NOALLOC_MAX_BUS buses and
 * DCOPF_PTDF_NOALLOC_MAX_LINE lines; larger ones get DCOPF_E_INVALID.
 * Every call on one device shares that workspace: calls that overlap on
 * one device (several host threads or streams) race and must be
 * serialised by the caller.  The call runs on the current device and
 * synchronises hip_stream before returning.                              */
#define DCOPF_PTDF_NOALLOC_MAX_BUS 2049
#define DCOPF_PTDF_NOALLOC_MAX_LINE 16384
dcopf_status dcopf_ptdf_noalloc(int32_t n_bus, int32_t n_line, const int32_t *fbus,
                                const int32_t *tbus, const double *b, int32_t slack,
                                void *hip_stream, double *H);

#ifdef __cplusplus
}
#endif

#endif /* DCOPF_PTDF_H */
