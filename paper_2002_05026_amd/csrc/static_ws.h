// The library's static device workspace (static_ws.hip) and the bind step it
// shares with d3m_factor_bind (capi.cpp).
#pragma once
#include <stddef.h>

#include "../../include/d3m.h"

namespace d3m {

// Whether generation gen is still the factor bound last to the static array
// of device dev.
bool static_ws_valid(int dev, unsigned long long gen);

// d3m_factor_bind on the workspace dev_ws; sdev >= 0 marks the factor as
// living in the static array of device sdev as generation sgen.
d3m_status bind_factor(d3m_plan plan, d3m_precision prec, void* dev_ws, size_t bytes, int32_t nrhs_max,
                       const d3m_options* opt, int sdev, unsigned long long sgen, d3m_factor* out);

}  // namespace d3m
