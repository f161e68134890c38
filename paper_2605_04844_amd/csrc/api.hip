// Status strings and version of libquadbox.
#include "qb_common.h"

extern "C" const char* qb_status_string(qb_status s)
{
    switch (s) {
        case QB_OK: return "ok";
        case QB_ERR_INVALID_ARG: return "invalid argument";
        case QB_ERR_CAPACITY: return "pair capacity exceeded";
        case QB_ERR_HIP: return "HIP runtime error";
        case QB_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

extern "C" int32_t qb_version(void) { return 101; }

extern "C" qb_status qb_check_capacity(int32_t count, const int64_t* num_pairs, const int64_t* capacities,
                                       int64_t* out_counts, qb_stream_t stream)
{
    if (count < 1 || count > (1 << 20) || !num_pairs || !capacities) return QB_ERR_INVALID_ARG;
    for (int32_t i = 0; i < count; ++i)
        if (capacities[i] < 0) return QB_ERR_INVALID_ARG;
    int64_t small[64];
    int64_t* host = out_counts ? out_counts : (count <= 64 ? small : nullptr);
    if (!host) return QB_ERR_INVALID_ARG;   // more than 64 counts need the caller's array
    hipStream_t s = qb_hip_stream(stream);
    if (hipMemcpyAsync(host, num_pairs, sizeof(int64_t) * (size_t)count, hipMemcpyDeviceToHost, s) != hipSuccess)
        return QB_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return QB_ERR_HIP;
    for (int32_t i = 0; i < count; ++i)
        if (host[i] > capacities[i]) return QB_ERR_CAPACITY;
    return QB_OK;
}
