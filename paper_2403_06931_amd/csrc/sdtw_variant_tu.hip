// sdtw_variant_tu.hip -- compiled once per forward tile variant, with
// -DSDTW_VARIANT_INDEX=i -DSDTW_R=.. -DSDTW_T=.. -DSDTW_W=.. -DSDTW_KS=.. -DSDTW_XL=..
// (taken by the build script from the list in sdtw_variants.inc).
#include "sdtw_variant.hpp"

#define SDTW_CAT2(a, b) a##b
#define SDTW_CAT(a, b) SDTW_CAT2(a, b)

sdtw::Variant SDTW_CAT(sdtw_variant_entry_, SDTW_VARIANT_INDEX)() {
  return sdtw::make_variant<SDTW_R, SDTW_T, SDTW_W, SDTW_KS, SDTW_XL>();
}
