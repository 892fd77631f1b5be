/*
 * bf_test.h -- test hooks of libbf.  Not for production use: they exist so
 * that the test suite can check host-visible pieces of the kernels and reach
 * code paths that production sizes reach only with very large inputs.  They
 * follow the conventions of bf.h (status returns, bf_last_error).
 */
#ifndef BF_TEST_H
#define BF_TEST_H

#include <stdint.h>

#include "bf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The Hann window of Eq. 3, W(u) = cos^2(pi u) for u < 1/2, as the gather
 * kernels evaluate it: the library's degree-6 polynomial in w = u^2 (the
 * same host/device function, evaluated on the host in FP32). */
double bf_test_hann_poly(double u2);

/* Cap on the frames one launch of bf_das_adjoint_frames takes (each gradient
 * of a stack goes in launches of at most `cap` frames; 0 = no cap, the
 * default: as many as the plan's partial-sum buffer holds).  Results do not
 * depend on it.  BF_ERR_SHAPE for cap < 0. */
int bf_test_set_stack_cap(bf_plan plan, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* BF_TEST_H */
