// Host build of the evaluator's binary32 transcendentals (gp_math.h), for
// testing them against the oracle on the CPU.
#include <stdint.h>

#include "gp_math.h"

namespace {
alignas(16) double g_tab[gpx::gmath::kTabSize];
bool g_ready = false;

template <int N>
void eval(int op, float (&a)[N]) {
    if (!g_ready) {
        gpx::gmath::tab_fill(g_tab, 0, 1);
        g_ready = true;
    }
    switch (op) {
        case 4: gpx::gmath::sincos_n<N>(a, false, g_tab, 0); break;
        case 5: gpx::gmath::sincos_n<N>(a, true, g_tab, 0); break;
        case 6: gpx::gmath::expc_n<N>(a, g_tab, 0); break;
        default: gpx::gmath::plog_n<N>(a, g_tab, 0); break;
    }
}
}  // namespace

extern "C" void gm_eval_n8(int op, const float* in, float* out, int64_t n) {
    for (int64_t i = 0; i + 8 <= n; i += 8) {
        float a[8];
        for (int j = 0; j < 8; j++) a[j] = in[i + j];
        eval<8>(op, a);
        for (int j = 0; j < 8; j++) out[i + j] = a[j];
    }
}

extern "C" void gm_eval(int op, const float* in, float* out, int64_t n) {
    for (int64_t i = 0; i < n; i++) {
        float a[1] = {in[i]};
        eval<1>(op, a);
        out[i] = a[0];
    }
}
