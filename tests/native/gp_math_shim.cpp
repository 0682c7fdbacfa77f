// Host build of the evaluator's binary32 transcendentals (gp_math.h), for
// testing them against the oracle on the CPU.
#include <stdint.h>

#include "gp_math.h"

extern "C" void gm_eval_n8(int op, const float* in, float* out, int64_t n) {
    for (int64_t i = 0; i + 8 <= n; i += 8) {
        float a[8];
        for (int j = 0; j < 8; j++) a[j] = in[i + j];
        switch (op) {
            case 4: gpx::gmath::sincos_n<8>(a, false, 0); break;
            case 5: gpx::gmath::sincos_n<8>(a, true, 0); break;
            case 6: gpx::gmath::expc_n<8>(a, 0); break;
            default: gpx::gmath::plog_n<8>(a, 0); break;
        }
        for (int j = 0; j < 8; j++) out[i + j] = a[j];
    }
}

extern "C" void gm_eval(int op, const float* in, float* out, int64_t n) {
    for (int64_t i = 0; i < n; i++) {
        const float a = in[i];
        switch (op) {
            case 4: out[i] = gpx::gmath::sin32(a); break;
            case 5: out[i] = gpx::gmath::cos32(a); break;
            case 6: out[i] = gpx::gmath::expc32(a); break;
            default: out[i] = gpx::gmath::plog32(a); break;
        }
    }
}
