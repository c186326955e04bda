/* Drives every entry point of the oracle over small and edge-case inputs
 * (empty, single, tie-heavy, subsets, non-finite values) so that a build
 * with the address and undefined-behaviour sanitizers can check its memory
 * accesses and arithmetic.  Built and run by tests/test_oracle_sanitized.py.
 * Prints "ok" and exits 0 when every call returns. */
#include "../oracle/gsoracle.c"

#include <stdio.h>
#include <stdlib.h>

static double* dalloc(int64_t n, double fill) {
    double* p = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) p[i] = fill + 1e-3 * (double)(i % 17) - 8e-3;
    return p;
}

static void make_groups(orc_group* G, int64_t n, const int* dims, int ng) {
    for (int g = 0; g < ng; ++g) {
        G[g].param = dalloc(n * dims[g], 0.3);
        G[g].grad = dalloc(n * dims[g], 1e-3);
        G[g].m = dalloc(n * dims[g], 1e-4);
        G[g].v = dalloc(n * dims[g], 1e-6);
        G[g].dim = dims[g];
        G[g].lr = 1e-2;
        G[g].dar_kind = g == 1 ? 2 : (g == 3 ? 1 : 0);
        G[g].dar_lambda = G[g].dar_kind ? 1e-3 : 0.0;
        G[g].dar_clip = 10.0;
        G[g].reg_mode = g % 3;
    }
}

static void free_groups(orc_group* G, int ng) {
    for (int g = 0; g < ng; ++g) {
        free(G[g].param);
        free((void*)G[g].grad);
        free(G[g].m);
        free(G[g].v);
    }
}

int main(void) {
    const int dims[5] = {3, 3, 4, 1, 48};
    const int ng = 5;
    orc_camera cam = {{1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 15}, 866.0f, 866.0f, 500.0f, 500.0f, 1000, 1000,
                      0.2f, 17.5f, 0.5f};
    orc_camera cams[3] = {cam, cam, cam};
    cams[1].view[3] = 2.0f;
    cams[2].view[11] = -1.0f;
    for (int64_t n = 0; n <= 70; n += (n < 3 ? 1 : 67)) {
        float* means = (float*)malloc(sizeof(float) * (size_t)(3 * n + 1));
        float* radius = (float*)malloc(sizeof(float) * (size_t)(n + 1));
        for (int64_t i = 0; i < 3 * n; ++i) means[i] = (float)((i * 37) % 23) - 11.0f;
        for (int64_t i = 0; i < n; ++i) radius[i] = 0.01f * (float)(i % 5);
        if (n > 2) means[4] = NAN;
        uint8_t* mask = (uint8_t*)malloc((size_t)n + 1);
        uint8_t* mask2 = (uint8_t*)malloc((size_t)n + 1);
        uint32_t* bits = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n + 1));
        int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
        orc_visibility(means, NULL, n, &cam, mask);
        orc_visibility(means, radius, n, &cam, mask2);
        orc_visibility_f64(means, radius, n, &cam, mask2);
        orc_visibility_multi(means, radius, n, cams, 3, mask2, bits);
        int64_t nv = orc_compact(mask, n, idx);
        (void)nv;
        for (int64_t i = 0; i < n; ++i) mask[i] = (uint8_t)((i * 7) % 3 == 0);

        orc_group G[5];
        make_groups(G, n, dims, ng);
        if (n > 2) ((double*)G[4].grad)[5] = NAN;
        int32_t* t = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
        int64_t* ids = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        for (int64_t i = 0; i < n; ++i) ids[i] = 3 * i + 1;
        orc_config cfg;
        memset(&cfg, 0, sizeof cfg);
        cfg.beta1 = 0.9; cfg.beta2 = 0.999; cfg.eps = 1e-15; cfg.reg_norm = 1e5;
        cfg.seed = 7; cfg.iteration = 3;
        cfg.rsr_enable = 1; cfg.rsr_alpha1 = 0.2; cfg.rsr_alpha2 = 0.04; cfg.rsr_ratio = 0.5;
        cfg.noise_enable = 1; cfg.noise_groups[0] = 0; cfg.noise_groups[1] = 1; cfg.noise_groups[2] = 2;
        cfg.noise_groups[3] = 3; cfg.noise_lr = 5.0; cfg.noise_k = 100.0; cfg.noise_t = 0.005;
        cfg.aiu_enable = 1; cfg.aiu_ratio = 0.5; cfg.aiu_scale = 0.5;
        orc_adamw_gs_step(G, ng, n, mask, t, &cfg);
        orc_adamw_gs_step_rows(G, ng, n, ids, mask, t, &cfg);
        orc_adamw_gs_step(G, ng, n, NULL, t, &cfg);
        orc_rsr_sample_mask(7, 3, ids, n, 0.3, mask2);
        orc_rsr_sample_mask(7, 3, NULL, n, 1.0, mask2);
        orc_aiu_sample_mask(7, 3, ids, n, 0.0, mask2);

        /* selection: tie-heavy keys, every k */
        float* key = (float*)malloc(sizeof(float) * (size_t)(n + 1));
        int64_t* sel = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        for (int64_t i = 0; i < n; ++i) key[i] = (float)((i * 5) % 4) - (i % 2 ? 0.0f : -0.0f);
        for (int64_t k = 0; k <= n; k += (n > 8 ? 7 : 1)) orc_select_smallest(key, n, k, sel);
        orc_select_smallest(key, n, n, sel);
        orc_reset_state(G, ng, sel, n / 2, t, 1);

        /* prune into a second set, then append clones of the first rows */
        orc_group D[5];
        make_groups(D, n, dims, ng);
        int32_t* t2 = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
        int64_t kept = orc_prune(G, D, ng, n, mask, t, t2);
        orc_group A[5];
        int64_t extra = 5;
        make_groups(A, n + extra, dims, ng);
        int32_t* t3 = (int32_t*)calloc((size_t)(n + extra) + 1, sizeof(int32_t));
        int64_t src[5] = {0, 0, 0, 0, 0};
        if (n > 0) orc_append(A, ng, n, src, extra, t3);
        (void)kept;

        double g3[3], out[3];
        double q[4] = {1, 2, 3, 4}, kap[3] = {0.1, -0.2, 0.3};
        orc_noise_gamma(7, 3, n, g3);
        orc_noise_displacement(q, kap, 0.4, 1.6e-4, &cfg, g3, out);
        (void)orc_reg_norm(1089480.0);
        (void)orc_bf16_rne(NAN);
        (void)orc_bf16_sr(INFINITY, 0xFFFFu);
        (void)orc_bf16_sr(-1.5f, 0x8000u);

        free_groups(G, ng); free_groups(D, ng); free_groups(A, ng);
        free(means); free(radius); free(mask); free(mask2); free(bits); free(idx); free(t); free(t2); free(t3);
        free(ids); free(key); free(sel);
    }
    printf("ok\n");
    return 0;
}
