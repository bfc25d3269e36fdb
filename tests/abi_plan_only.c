/* The C ABI used from plain C (C11, no C++): a plan-only session (no device)
 * goes through the whole modifier and update cycle, and every call reports
 * its status.  Prints one line per check; exits non-zero on the first
 * failure. */
#include <stdio.h>
#include <string.h>

#include "qtask.h"

#define CHECK(cond, what)                                  \
    do {                                                   \
        if (!(cond)) {                                     \
            printf("FAIL %s (line %d)\n", what, __LINE__); \
            return 1;                                      \
        }                                                  \
        printf("ok %s\n", what);                           \
    } while (0)

int main(int argc, char **argv) {
    const char *dot = argc > 1 ? argv[1] : "plan.dot";
    qtask_opts o;
    memset(&o, 0, sizeof o);
    CHECK(qtask_opts_default(&o) == QTASK_OK, "defaults");
    o.device = QTASK_DEVICE_NONE;
    o.tile_bits = 5;
    o.low_bits = 2;
    o.ckpt_interval = 2;
    qtask_t h = NULL;
    CHECK(qtask_create(6, QTASK_C128, &o, &h) == QTASK_OK && h != NULL, "create");

    /* three levels: H on every qubit, a CX ladder, RZ on qubit 5 */
    qtask_level_t lv[3];
    qtask_level_t after = QTASK_FRONT;
    for (int i = 0; i < 3; ++i) {
        CHECK(qtask_insert_level(h, after, &lv[i]) == QTASK_OK, "insert level");
        after = lv[i];
    }
    qtask_gate_t g;
    for (int32_t q = 0; q < 6; ++q) CHECK(qtask_insert_gate(h, lv[0], QTASK_H, &q, 1, NULL, 0, &g) == QTASK_OK, "H");
    for (int32_t q = 0; q + 1 < 6; q += 2) {
        const int32_t qs[2] = {q, q + 1};
        CHECK(qtask_insert_gate(h, lv[1], QTASK_CX, qs, 2, NULL, 0, &g) == QTASK_OK, "CX");
    }
    const int32_t q5 = 5;
    const double theta = 0.25;
    qtask_gate_t rz;
    CHECK(qtask_insert_gate(h, lv[2], QTASK_RZ, &q5, 1, &theta, 1, &rz) == QTASK_OK, "RZ");
    /* a second gate on qubit 5 in the same level conflicts and changes nothing */
    CHECK(qtask_insert_gate(h, lv[2], QTASK_X, &q5, 1, NULL, 0, &g) == QTASK_E_CONFLICT, "conflict rejected");
    /* a wrong parameter count is an argument error */
    CHECK(qtask_insert_gate(h, lv[2], QTASK_RZ, &q5, 1, NULL, 0, &g) == QTASK_E_ARG, "missing angle rejected");
    uint64_t n_gates = 0, n_levels = 0;
    CHECK(qtask_num_gates(h, &n_gates) == QTASK_OK && n_gates == 10, "ten gates");
    CHECK(qtask_num_levels(h, &n_levels) == QTASK_OK && n_levels == 3, "three levels");

    qtask_stats st;
    memset(&st, 0, sizeof st);
    st.struct_size = sizeof st;
    CHECK(qtask_update_state(h) == QTASK_OK, "first update");
    CHECK(qtask_last_update_stats(h, &st) == QTASK_OK && st.mode == 1 && st.levels_total == 3, "full mode");

    /* edit the last level: the update restarts at a checkpoint before it */
    CHECK(qtask_remove_gate(h, rz) == QTASK_OK, "remove RZ");
    CHECK(qtask_update_state(h) == QTASK_OK, "incremental update");
    CHECK(qtask_last_update_stats(h, &st) == QTASK_OK && (st.mode == 2 || st.mode == 3) && st.first_level >= 2,
          "restart after the checkpoint");
    CHECK(qtask_update_state(h) == QTASK_OK && qtask_last_update_stats(h, &st) == QTASK_OK && st.mode == 0,
          "nothing left to do");

    /* a plan-only session computes no amplitudes */
    double amp[2];
    CHECK(qtask_read_amplitudes(h, 0, 1, amp) == QTASK_E_UNSUPPORTED, "no amplitudes without a device");
    CHECK(qtask_dump_plan(h, dot) == QTASK_OK, "dump the plan as DOT");
    CHECK(strlen(qtask_status_string(QTASK_E_CONFLICT)) > 0, "status string");
    CHECK(qtask_destroy(h) == QTASK_OK, "destroy");
    return 0;
}
