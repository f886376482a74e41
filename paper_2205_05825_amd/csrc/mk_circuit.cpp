// Netlist builders and circuit evaluation (placeholder until they land).
#include "mk_internal.h"

using namespace mk;

extern "C" {

int mk_eval_circuit(mk_ctx *, const mk_circuit *, const uint32_t *, uint32_t *, size_t, size_t,
                    int, void *) {
    return fail(MK_EINVAL, "mk_eval_circuit not built yet");
}

int mk_build_operator(int, int, mk_gate *, int32_t *, int32_t *, int32_t *, int32_t *) {
    return fail(MK_EINVAL, "mk_build_operator not built yet");
}

}
