// internal.h -- functions shared between the translation units of libhers
// (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/hers.h"

namespace hers {
// hers_api.cpp
void set_last_error(const std::string& msg);   // the message hers_last_error() returns on this thread
int ctx_device(const hers_ctx* ctx);
size_t search_ws_block_bytes(const hers_ctx* ctx);   // search workspace per gallery block
int search_impl(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m, int32_t d,
                const uint32_t* probe_dev, uint64_t probe_words, uint64_t* scores_dev, void* work_dev,
                size_t work_bytes, void* stream, bool overlap);
int encrypt_probe_prechecked(hers_ctx* ctx, const int32_t* query, int32_t d, uint64_t seed, uint32_t* probe_dev,
                             void* work_dev, size_t work_bytes, hipStream_t s);   // query: host, range checked
// noalloc.hip: resolves this device's copy of the static scratch array (call
// with `device` current)
int scratch_setup(int device);
}  // namespace hers
