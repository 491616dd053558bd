// Host-side access to the PTC network for the FGCR solver.
#pragma once

#include "wd_internal.h"

namespace wd {
// z = N(r): F32 full fields; runs on stream st.
wd_status ptc_apply(const wd_ptc *n, const void *in, void *out, hipStream_t st);
const wd_gauge *ptc_gauge(const wd_ptc *n);
}  // namespace wd
