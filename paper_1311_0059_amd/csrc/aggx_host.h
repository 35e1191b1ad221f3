// Host-side helpers of the runtime shared with the other host entry points
// (internal; not part of the public C ABI).
#pragma once

#include "../../include/aggx.h"
#include "aggx_internal.h"

namespace aggx {
// AGG_OK, or the status agg_create gives a malformed spec.
agg_status spec_check(const agg_spec *s);
// The kernels' view of a checked spec.
KSpec spec_kernels(const agg_spec &s);
// Launch shape of the on-chip engine for n records with about G groups (aligned16:
// the records start on a 16-byte boundary); false when they need more key
// classes than it takes.
bool onchip_shape(const KSpec &ks, uint64_t n, double G, bool aligned16, OnchipPlan *op);
}  // namespace aggx
