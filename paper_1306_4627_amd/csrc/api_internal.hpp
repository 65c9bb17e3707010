// api_internal.hpp -- library-internal batch interface used by the request
// server: batches that run on a given stream, take their device memory from
// a caller's arena, and are completed by polling instead of waiting.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "lcs.h"

namespace lcs {

struct BatchHooks {
    hipStream_t stream = nullptr;                          // uploads and kernels go here
    void *(*alloc)(void *user, size_t bytes) = nullptr;    // device memory instead of hipMalloc
    void (*release)(void *user, void *ptr) = nullptr;      // returns it
    void *user = nullptr;
    // device bytes the batch may hold at most (0: no limit known); a
    // traceback batch whose full history would not fit runs in rounds
    size_t avail = 0;
};

// lcs_batch_create with hooks (hooks may be null).
lcs_status batch_create(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                        const lcs_alphabet *alphabet, uint32_t flags, const lcs_tuning *tuning,
                        const BatchHooks *hooks, lcs_batch **out);

// Enqueue one pass (kernels launched directly) and return at once.
lcs_status batch_launch(lcs_batch *b);

// 1 when the last pass has finished, 0 while it runs, a negative status on
// a HIP failure.
int batch_query(lcs_batch *b);

// After batch_query returned 1: the lengths (input order) and, for batches
// with LCS_WANT_TRACEBACK, each pair's LCS string.
lcs_status batch_results(lcs_batch *b, std::vector<uint64_t> &lens,
                         std::vector<std::vector<uint8_t>> *strings);

// Validate an alphabet and a pair's bytes against it; *sigma = its size.
lcs_status alphabet_check(const lcs_alphabet *a, const uint8_t *x, uint64_t m, const uint8_t *y,
                          uint64_t n, int *sigma);

// Device of a context.
int ctx_device(lcs_ctx *ctx);

// Reserve device memory from a context's budget (*bytes == 0: half of what
// is left), allocated at once; *bytes receives the size.
lcs_status ctx_reserve(lcs_ctx *ctx, size_t *bytes, void **mem);
void ctx_unreserve(lcs_ctx *ctx, void *mem, size_t bytes);

// The autotuner's cached tuning for a batch of this shape, if any.
bool tuning_cached(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count, int sigma, uint32_t flags,
                   lcs_tuning *out);

}  // namespace lcs
