/* The C ABI from plain C99: the headers compile as C, the library links, and
 * the struct layouts it reports are compared with the Python binding's by
 * tests/test_abi.py.  Makes no call that touches a device. */
#include <stddef.h>
#include <stdio.h>

#include "lrep.h"
#include "lrep_testing.h"

int main(void) {
    if (lrep_version() <= 0) return 1;
    if (lrep_solve(NULL, 1, 1, 1, 1e-8, NULL, NULL, NULL, NULL, 1, NULL) != LREP_EINVAL) return 2;
    if (lrep_set_metric(NULL, 1, NULL, 0) != LREP_EINVAL) return 3;
    if (lrep_strerror(LREP_EINVAL) == NULL) return 4;
    printf("opts %zu stats %zu request %zu graphs %zu precision %zu init_U %zu\n", sizeof(lrep_solve_opts_t),
           sizeof(lrep_stats_t), sizeof(lrep_request_t), offsetof(lrep_solve_opts_t, graphs),
           offsetof(lrep_solve_opts_t, precision), offsetof(lrep_solve_opts_t, init_U));
    return 0;
}
