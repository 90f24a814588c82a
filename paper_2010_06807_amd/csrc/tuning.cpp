// Process-wide kernel dispatch thresholds (the tile and block-size schedule).
#include "common.hpp"

namespace spaqr {

namespace {
constexpr spaqr_tuning kDefault = {1024, 1024, 1024, 1, 1, 64, 64, 1, 2, 2};
spaqr_tuning g_tuning = kDefault;

bool valid(const spaqr_tuning& t) {
  auto cls = [](int v) { return v == 0 || v == 16 || v == 32 || v == 64; };
  return (t.qr_reg_max_rows == 256 || t.qr_reg_max_rows == 512 || t.qr_reg_max_rows == 1024) &&
         t.split_rows >= 1 && t.split_cols >= 1 && (t.cpqr_reg == 0 || t.cpqr_reg == 1) &&
         (t.cpqr_coop == 0 || t.cpqr_coop == 1) && cls(t.scale_small) &&
         cls(t.iface_dense) && (t.trail_mfma == 0 || t.trail_mfma == 1) && (t.cpqr_dd >= 0 && t.cpqr_dd <= 2) &&
         (t.cpqr_team >= 0 && t.cpqr_team <= 2);
}
}  // namespace

const spaqr_tuning& tuning() { return g_tuning; }

}  // namespace spaqr

extern "C" {

spaqr_status spaqr_set_tuning(const spaqr_tuning* t) {
  if (!t) {
    spaqr::g_tuning = spaqr::kDefault;
    return SPAQR_OK;
  }
  if (!spaqr::valid(*t)) return SPAQR_EINVAL;
  spaqr::g_tuning = *t;
  return SPAQR_OK;
}

spaqr_status spaqr_get_tuning(spaqr_tuning* t) {
  if (!t) return SPAQR_EINVAL;
  *t = spaqr::g_tuning;
  return SPAQR_OK;
}

}  // extern "C"
