/* Compiles include/fnlsim.h as C11 and calls the library's validation paths,
 * which run before any HIP call, so this program needs no GPU.  Exit status 0
 * when every check holds; the first failing check is printed. */
#include <stdio.h>
#include <string.h>

#include "fnlsim.h"

#define CHECK(cond)                                                      \
    do {                                                                 \
        if (!(cond)) {                                                   \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                    \
        }                                                                \
    } while (0)

int main(void)
{
    enum { L = 4, N = 3 };
    double r[N], w[N], filt[(L + 1) * N * N], alpha[(L + 1) * N], beta[(L + 1) * N];
    for (int i = 0; i < N; i++) {
        r[i] = 13000.0 + 100.0 * i;
        w[i] = 100.0;
    }
    memset(filt, 0, sizeof filt);
    for (int l = 0; l <= L; l++)
        for (int i = 0; i < N; i++) filt[(l * N + i) * N + i] = 1.0;
    for (int k = 0; k < (L + 1) * N; k++) alpha[k] = beta[k] = 1.0;

    sim_ctx *ctx = NULL;
    sim_opts o;
    memset(&o, 0, sizeof o);

    /* bad arguments are rejected with SIM_EINVAL and a message */
    CHECK(sim_init(NULL, L, N, r, w, filt, alpha, beta, &o) == SIM_EINVAL);
    CHECK(sim_init(&ctx, 0, N, r, w, filt, alpha, beta, &o) == SIM_EINVAL && ctx == NULL);
    CHECK(sim_init(&ctx, L, N, r, w, NULL, alpha, beta, &o) == SIM_EINVAL && ctx == NULL);
    o.precision = 9;
    CHECK(sim_init(&ctx, L, N, r, w, filt, alpha, beta, &o) == SIM_EINVAL && ctx == NULL);
    o.precision = SIM_FP64;
    o.ring_shells = 2;
    CHECK(sim_init(&ctx, L, N, r, w, filt, alpha, beta, &o) == SIM_EINVAL && ctx == NULL);
    o.ring_shells = 0;
    o.n_phi = 3 * L - 1;
    CHECK(sim_init(&ctx, L, N, r, w, filt, alpha, beta, &o) == SIM_EINVAL && ctx == NULL);
    const char *msg = sim_last_error(NULL);
    CHECK(msg != NULL && strlen(msg) > 0 && strcmp(msg, "no error") != 0);

    /* calls on a null context */
    CHECK(sim_destroy(NULL) == SIM_OK);
    CHECK(sim_forward(NULL, NULL, 1, NULL, NULL, NULL, NULL, NULL) == SIM_EINVAL);
    CHECK(sim_tqu_maps(NULL, NULL, NULL, 1, NULL) == SIM_EINVAL);
    CHECK(sim_ksw_cubic(NULL, NULL, NULL, 1, NULL) == SIM_EINVAL);
    sim_info info;
    CHECK(sim_get_info(NULL, &info) == SIM_EINVAL);
    CHECK(sim_batch_destroy(NULL) == SIM_OK);
    printf("C ABI checks passed\n");
    return 0;
}
