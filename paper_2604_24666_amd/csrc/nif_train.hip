// Training: multi-task loss, hand-written backward and Adam.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "nif_internal.hpp"
#include "nif_net.hpp"

namespace nif {

int model_reserve(nif_model* m, int64_t B) {
    if (B <= m->max_batch) return NIF_OK;
    for (float** p : {&m->dz, &m->acts, &m->delta, &m->delta1})
        if (*p) { (void)hipFree(*p); *p = nullptr; }
    m->max_batch = 0;
    const int64_t hw = m->desc.hidden_width, nh = m->desc.hidden_layers;
    const struct { float** p; int64_t n; } a[] = {{&m->dz, B * 16}, {&m->acts, B * hw * nh}, {&m->delta, B * hw * nh}, {&m->delta1, B * hw}};
    for (auto& x : a)
        if (hipMalloc((void**)x.p, sizeof(float) * (size_t)std::max<int64_t>(x.n, 1)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(NIF_E_OOM, "training scratch allocation failed");
        }
    m->max_batch = B;
    return NIF_OK;
}

int backward_launch(nif_model*, const float*, const float*, int64_t, const float*, int32_t, float*, float*, int32_t,
                    hipStream_t) {
    return fail(NIF_E_UNSUPPORTED, "backward not built yet");
}

int train_step_launch(nif_model*, const nif_batch*, int64_t, const nif_train_cfg*, float*, hipStream_t) {
    return fail(NIF_E_UNSUPPORTED, "train step not built yet");
}

}  // namespace nif
