/* Stand-in for <hip/hip_runtime_api.h> in the host build: the stream
 * handle type that the C ABI's declarations name. */
#pragma once
typedef struct ihipStream_t *hipStream_t;
