// Internal helpers of runtime.cpp used by the serving core (server.cpp).
#pragma once

#include <cstddef>
#include <string>

#include <hip/hip_runtime_api.h>

#include "nao.h"

namespace nao {

// Device allocation through a context (counted against its HBM budget).
nao_status ctx_alloc(nao_ctx c, size_t bytes, void** out);
void ctx_free(nao_ctx c, void* p, size_t bytes);
hipStream_t ctx_stream(nao_ctx c);
int ctx_device(nao_ctx c);
void ctx_set_error(nao_ctx c, const std::string& msg);
size_t system_device_bytes(nao_system s);

}  // namespace nao
