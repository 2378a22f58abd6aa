// Context-based pipeline entry points (placeholder until the runtime lands).
#include "common.hpp"

using namespace nc;

extern "C" {
nc_status nc_create(const nc_config*, const float*, nc_ctx**) {
  return guard([&] { fail(NC_E_STATE, "not implemented"); });
}
void nc_destroy(nc_ctx*) {}
nc_status nc_streams_reset(nc_ctx*, uint32_t, uint32_t) {
  return guard([&] { fail(NC_E_STATE, "not implemented"); });
}
nc_status nc_calibrate_fp8(nc_ctx*, const int32_t*, size_t) {
  return guard([&] { fail(NC_E_STATE, "not implemented"); });
}
nc_status nc_probs_for_context(nc_ctx*, uint32_t, const int32_t*, size_t, float*, nc_probe*) {
  return guard([&] { fail(NC_E_STATE, "not implemented"); });
}
nc_status nc_mix_update(nc_ctx*, uint32_t, int32_t) {
  return guard([&] { fail(NC_E_STATE, "not implemented"); });
}
nc_status nc_encode_stream(nc_ctx*, uint32_t, const int32_t* const*, const size_t*,
                           uint8_t* const*, const size_t*, size_t*, uint64_t*) {
  return guard([&] { fail(NC_E_STATE, "not implemented"); });
}
nc_status nc_decode_stream(nc_ctx*, uint32_t, const uint8_t* const*, const size_t*,
                           const size_t*, int32_t* const*) {
  return guard([&] { fail(NC_E_STATE, "not implemented"); });
}
nc_status nc_get_stats(const nc_ctx*, nc_stats*) {
  return guard([&] { fail(NC_E_STATE, "not implemented"); });
}
nc_status nc_ensemble_forward(const float*, const float*, const float*, const float*,
                              const int32_t*, uint32_t, uint32_t, uint32_t, float*, float*,
                              float*, void*) {
  return guard([&] { fail(NC_E_STATE, "not implemented"); });
}
nc_status nc_ensemble_backward(const float*, float*, float*, const float*, const int32_t*,
                               const float*, uint32_t, uint32_t, uint32_t, float, float*, float*,
                               void*) {
  return guard([&] { fail(NC_E_STATE, "not implemented"); });
}
}
