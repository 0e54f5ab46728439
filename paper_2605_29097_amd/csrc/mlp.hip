// SDF network: placeholder entry points until the MFMA kernels land.
#include "rfvr_impl.hpp"

using namespace rfvr;

extern "C" {

int64_t rfvr_mlp_param_count(const rfvr_mlp* net) {
    if (!net || net->n_layers < 1 || net->width < 1 || net->head_layers < 1 || net->head_width < 1 ||
        net->pe_octaves < 0)
        return -1;
    const int64_t in0 = 3 + 6 * (int64_t)net->pe_octaves;
    int64_t n = (int64_t)net->width * in0 + net->width;
    n += (int64_t)(net->n_layers - 1) * ((int64_t)net->width * net->width + net->width);
    n += net->width + 1;
    n += (int64_t)net->head_width * net->width + net->head_width;
    n += (int64_t)(net->head_layers - 1) * ((int64_t)net->head_width * net->head_width + net->head_width);
    n += net->head_width + 1;
    return n;
}

size_t rfvr_mlp_forward_ws_bytes(const rfvr_mlp*, int64_t) { return 0; }
size_t rfvr_mlp_backward_ws_bytes(const rfvr_mlp*, int64_t) { return 0; }
int rfvr_mlp_forward(const rfvr_mlp*, const float*, int64_t, float*, float*, float*, void*, size_t, void*) {
    set_error("rfvr_mlp_forward: not built yet");
    return RFVR_E_UNSUPPORTED;
}
int rfvr_mlp_backward(const rfvr_mlp*, const float*, int64_t, const float*, const float*, const float*,
                      uint32_t, float*, void*, size_t, void*) {
    set_error("rfvr_mlp_backward: not built yet");
    return RFVR_E_UNSUPPORTED;
}
}
