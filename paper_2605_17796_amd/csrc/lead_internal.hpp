// Library-internal entry points shared between the C ABI translation units.
#pragma once
#include <cstdint>

#include "../../include/lead.h"

namespace lead {

// A new decoder with the same code, check type, parameters and schedule as
// `src`, sized for `max_shots` shots.
lead_status clone_decoder(const lead_decoder *src, int64_t max_shots, lead_decoder **out);
// Code length and number of checks of a decoder.
void decoder_shape(const lead_decoder *d, int *n, int *m);
// Device bytes a decoder holds (tables, workspace and the buffers it has
// allocated so far).
int64_t decoder_device_bytes(const lead_decoder *d);
// Records a failure message (returned by lead_last_error on this thread).
lead_status set_error(lead_status s, const char *msg);

}  // namespace lead
