// Library-internal calls between the translation units of libhho.so (not part of the C ABI).
#pragma once

#include <cstddef>
#include <string>

#include "../../include/hho.h"

namespace hho {

// Device ordinal of a context.
int ctx_device(const hho_ctx *ctx);

// Record an error message on a context (returned by hho_last_error).
void ctx_set_error(hho_ctx *ctx, const std::string &msg);

// Energy of every shot's current state into out[n_shots] (device memory), with the per-block
// partial sums in part[0 .. n_blocks * n_shots) (device memory, `cap` doubles).  Enqueued on the
// context's stream: no allocation, no synchronisation.  ARG (nothing launched) when the partial
// sums need more than `cap` doubles.
hho_status energy_into(hho_ctx *ctx, double *part, size_t cap, double *out);

// Set-up of the no-allocation entry points on `device` (noalloc.hip): resolves the device address
// of the library's static scratch array once per device.  Returns "" or an error message.
std::string noalloc_init(int device);

}  // namespace hho
