// sdtw_variant.hpp -- one compiled forward tile variant: its shape and the
// kernel entry points for each cost kind and checkpoint mode, its pruned,
// binary16 and uint8-code forms.
#pragma once

#include "sdtw_fwd.hpp"

namespace sdtw {

struct Variant {
  int R, T, W, KS, XL;
  const void* plain[2][2];        // [cost kind][checkpoint]
  const void* persistent[2][2];
  const void* half[2];            // [cost kind]: binary16, two queries per lane row
  const void* pruned[2];          // squared cost with early pruning: [plain, persistent]
  const void* u8;                 // integer DP on uint8 codes
  int lds_bytes;
};

template <int R, int T, int W, int KS, int XL>
Variant make_variant() {
  Variant v;
  v.R = R;
  v.T = T;
  v.W = W;
  v.KS = KS;
  v.XL = XL;
  v.plain[0][0] = reinterpret_cast<const void*>(&sdtw_fwd_kernel<R, T, W, KS, XL, 0, false>);
  v.plain[0][1] = reinterpret_cast<const void*>(&sdtw_fwd_kernel<R, T, W, KS, XL, 0, true>);
  v.plain[1][0] = reinterpret_cast<const void*>(&sdtw_fwd_kernel<R, T, W, KS, XL, 1, false>);
  v.plain[1][1] = reinterpret_cast<const void*>(&sdtw_fwd_kernel<R, T, W, KS, XL, 1, true>);
  v.persistent[0][0] = reinterpret_cast<const void*>(&sdtw_fwd_persistent_kernel<R, T, W, KS, XL, 0, false>);
  v.persistent[0][1] = reinterpret_cast<const void*>(&sdtw_fwd_persistent_kernel<R, T, W, KS, XL, 0, true>);
  v.persistent[1][0] = reinterpret_cast<const void*>(&sdtw_fwd_persistent_kernel<R, T, W, KS, XL, 1, false>);
  v.persistent[1][1] = reinterpret_cast<const void*>(&sdtw_fwd_persistent_kernel<R, T, W, KS, XL, 1, true>);
  v.pruned[0] = reinterpret_cast<const void*>(&sdtw_fwd_kernel<R, T, W, KS, XL, kPruned, false>);
  v.pruned[1] = reinterpret_cast<const void*>(&sdtw_fwd_persistent_kernel<R, T, W, KS, XL, kPruned, false>);
  v.u8 = reinterpret_cast<const void*>(&sdtw_fwd_u8_kernel<R, T, W, KS, XL>);
  v.half[0] = reinterpret_cast<const void*>(&sdtw_fwd16_kernel<R, T, W, KS, XL, 0>);
  v.half[1] = reinterpret_cast<const void*>(&sdtw_fwd16_kernel<R, T, W, KS, XL, 1>);
  v.lds_bytes = (int)(sizeof(float) * FwdShape<R, T, W, KS, XL>::LDS_FLOATS);
  return v;
}

}  // namespace sdtw

// Entry point of variant i, defined in the translation unit built for it.
#define SDTW_DECLARE_VARIANT(i, R, T, W, KS, XL) sdtw::Variant sdtw_variant_entry_##i();
