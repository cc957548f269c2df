// The explicit thermal update of one cell, shared by every stencil kernel
// (direct, LDS tile, vector rows, many-grid, and the surrogate's checks and
// fallback), so all of them round identically.
//   T' = T + c*(P + (Tn+Ts-2T)/Ry + (Te+Tw-2T)/Rx [+ (Tu+Td-2T)/Rz] + (Tamb-T)/Rz)
// evaluated as one fixed chain of fused multiply-adds with the coefficients
// c, c/Rx, c/Ry, c/Rz pre-rounded to float.
#pragma once

#include "kb_internal.h"

namespace kb {

__device__ __forceinline__ float heat_update(float t, float tn, float ts, float tw, float te, float p,
                                             const HeatCoef &k) {
  float dns = (tn + ts) - (t + t);
  float dew = (te + tw) - (t + t);
  float acc = k.cz * (k.Tamb - t);
  acc = fmaf(k.cx, dew, acc);
  acc = fmaf(k.cy, dns, acc);
  acc = fmaf(k.cP, p, acc);
  return t + acc;
}

__device__ __forceinline__ float heat3d_update(float t, float tn, float ts, float tw, float te, float tu,
                                               float td, float p, bool has_p, const HeatCoef &k) {
  float dns = (tn + ts) - (t + t);
  float dew = (te + tw) - (t + t);
  float dud = (tu + td) - (t + t);
  float acc = k.cz * (k.Tamb - t);
  acc = fmaf(k.cx, dew, acc);
  acc = fmaf(k.cz, dud, acc);
  acc = fmaf(k.cy, dns, acc);
  if (has_p) acc = fmaf(k.cP, p, acc);
  return t + acc;
}

}  // namespace kb
