// Context management and status strings of the C ABI.
#include "common.hpp"

#include <stdlib.h>

extern "C" const char* rbf_status_string(rbf_status s) {
    switch (s) {
        case RBF_OK: return "ok";
        case RBF_EINVAL: return "invalid argument";
        case RBF_ETOOFEW: return "stencil size larger than the node count";
        case RBF_EDIM: return "dimension must be 2 or 3";
        case RBF_EWORKSPACE: return "workspace too small";
        case RBF_EHIP: return "HIP runtime error";
        case RBF_EUNSUPPORTED: return "system size not compiled";
        default: return "unknown status";
    }
}

extern "C" rbf_status rbf_ctx_create(rbf_ctx** ctx, int device, void* hip_stream) {
    if (!ctx) return RBF_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return RBF_EHIP;
    if (device < 0 || device >= count) return RBF_EINVAL;
    {
        // resolve this device's copy of the no-allocation scratch with the device current
        int prev = 0;
        if (hipGetDevice(&prev) != hipSuccess) return RBF_EHIP;
        if (hipSetDevice(device) != hipSuccess) return RBF_EHIP;
        const rbf_status st = rbf_select_scratch_init(device);
        if (hipSetDevice(prev) != hipSuccess) return RBF_EHIP;
        if (st != RBF_OK) return st;
    }
    rbf_ctx* c = (rbf_ctx*)calloc(1, sizeof(rbf_ctx));
    if (!c) return RBF_EINVAL;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *ctx = c;
    return RBF_OK;
}

extern "C" rbf_status rbf_ctx_set_stream(rbf_ctx* ctx, void* hip_stream) {
    if (!ctx) return RBF_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return RBF_OK;
}

extern "C" rbf_status rbf_ctx_destroy(rbf_ctx* ctx) {
    if (!ctx) return RBF_EINVAL;
    if (ctx->mlp_params) {
        if (hipSetDevice(ctx->device) == hipSuccess) (void)hipFree(ctx->mlp_params);
    }
    free(ctx);
    return RBF_OK;
}
