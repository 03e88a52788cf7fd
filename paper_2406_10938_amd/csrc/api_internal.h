// Internal interface between the query orchestration (detlsh_api.cpp) and the
// serving loop (serve.cpp).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "detlsh.h"

// Sets the calling thread's detlsh_last_error message; returns s.
detlsh_status dl_error(detlsh_status s, const char* msg);

bool dl_is_device_ptr(const void* p);
int dl_index_device(detlsh_index ix);
int32_t dl_index_dim(detlsh_index ix);
int32_t dl_index_lk(detlsh_index ix);    // L*K
int64_t dl_index_n(detlsh_index ix);

// Checks the scalar arguments of a query of nq rows exactly as detlsh_query
// does; *bytes_one_pass (optional) receives the arena size that runs all nq
// queries in one pass, including one query of either fallback.
detlsh_status dl_query_check(detlsh_index ix, int64_t nq, int32_t k, double c, double beta,
                             const detlsh_query_opts* opts, size_t* bytes_one_pass);

// detlsh_query inside the caller's device arena [arena, arena + arena_bytes):
// no device memory is allocated or freed.  Runs in as many passes as the arena
// requires; ENOMEM if it cannot hold one query.  Synchronises `st`.
detlsh_status dl_query_in_arena(detlsh_index ix, const float* Q, int64_t nq, int32_t k, double c, double beta,
                                const detlsh_query_opts* opts, int64_t* out_ids, float* out_dists, void* arena,
                                size_t arena_bytes, hipStream_t st);
