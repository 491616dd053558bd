// Host-side access to the PTC network for the FGCR solver.
#pragma once

#include "wd_internal.h"

namespace wd {
// z = N(r): F32 full fields; runs on stream st.
wd_status ptc_apply(const wd_ptc *n, const void *in, void *out, hipStream_t st);
// out_e = [N (in_e, 0)]_e: F32 half fields (even parity); runs on stream st.
wd_status ptc_apply_even(const wd_ptc *n, const void *in_even, wd_prec pin, void *out_even, wd_prec pout,
                         hipStream_t st);
const wd_gauge *ptc_gauge(const wd_ptc *n);
}  // namespace wd
