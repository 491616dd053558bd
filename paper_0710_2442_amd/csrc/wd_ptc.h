// Host-side access to the PTC network for the FGCR solver.
#pragma once

#include "wd_internal.h"

namespace wd {
// z = N(r): F32 full fields; runs on stream st.
wd_status ptc_apply(const wd_ptc *n, const void *in, void *out, hipStream_t st);
// out_e = [N (in_e, 0)]_e: half fields (even parity) in pin / pout (FP32 or
// BF16); runs on stream st.
wd_status ptc_apply_even(const wd_ptc *n, const void *in_even, wd_prec pin, void *out_even, wd_prec pout,
                         hipStream_t st);
// The same with FP16 products and FP32 sums: in_even a BF16 half field,
// norm2 -> |in_even|^2 on the device; needs BF16 activations.
wd_status ptc_apply_even_h(const wd_ptc *n, const void *in_even, void *out_even, wd_prec pout, const double *norm2,
                           hipStream_t st);
// The same on the matrix cores (BF16 operands, FP32 sums); FP32 input is
// rounded to BF16 first.  Needs BF16 activations.
wd_status ptc_apply_even_b(const wd_ptc *n, const void *in_even, wd_prec pin, void *out_even, wd_prec pout,
                           hipStream_t st);
const wd_gauge *ptc_gauge(const wd_ptc *n);
wd_prec ptc_act(const wd_ptc *n);
}  // namespace wd
