"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a plain C
driver, built with the oracle source, runs a short simulation that touches
every subsystem (emission, push, collisions, the Langevin window, masked
space charge, the adaptive step, snapshots, exits) on a small ring grid.
Any out-of-bounds access, leak or undefined operation fails the test."""
import os
import subprocess

DRIVER = r'''
#include "mc_oracle.h"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
int main(void) {
    const int nr = 24, nz = 96;
    const double h = 5e-5, R = (nr - 1) * h, L = (nz - 1) * h;
    const size_t nn = (size_t)nr * nz;
    double *phi = calloc(nn, 8), *rf = calloc(nn, 8), *uz = calloc(nn, 8), *p = calloc(nn, 8), *t = calloc(nn, 8);
    unsigned char *mask = calloc(nn, 1);
    for (int j = 0; j < nz; ++j)
        for (int i = 0; i < nr; ++i) {
            size_t o = (size_t)j * nr + i;
            double z = j * h, r = i * h;
            phi[o] = -20.0 * z / L + 5.0 * exp(-((r - R / 2) * (r - R / 2) + (z - L / 2) * (z - L / 2)) / 1e-7);
            rf[o] = exp(-((r - R / 2) * (r - R / 2) + (z - L / 3) * (z - L / 3)) / 1e-7);
            uz[o] = 300.0 * exp(-z / L);
            p[o] = 2e3 * exp(-3.0 * z / L);
            t[o] = 300.0;
            if (i >= nr / 2 && i <= nr / 2 + 2 && abs(j - nz / 2) <= 2) mask[o] = 1;
        }
    orc_sim *s = orc_create(7);
    if (orc_load_fields(s, nr, nz, h, h, phi, NULL, rf, NULL, uz, p, t, mask)) return 2;
    orc_ion ion = {500.0, 1, 2e-18, 150, 1100.0, -1.0, 300.0, 1, 100e3, -80.0};
    if (orc_define_ion(s, &ion) < 0) return 3;
    orc_operating op;
    memset(&op, 0, sizeof(op));
    op.dt = 1e-9; op.v_rf = 50.0; op.f_rf = 1e6; op.gas_mass_da = 28.0134; op.collisions_on = 1;
    op.sc_on = 1; op.sc_every = 3; op.z_det = L; op.r_det = R; op.d_hit = 1e-5; op.exit_bin_dt = 1e-8;
    op.n_exit_bins = 50; op.langevin_on = 1; op.lv_z_lo = 0.0; op.lv_z_hi = L / 4; op.lv_switch = 0.05;
    op.sc_mask = 1; op.sample_every = 4; op.sample_stride = 3; op.adaptive = 1; op.lv_dt_max = 5e-10;
    if (orc_set_operating(s, &op)) return 4;
    orc_source src;
    memset(&src, 0, sizeof(src));
    src.kind = 2; src.ion = 0; src.current_a = 5e-9; src.weight = 50.0; src.n_total = 3000;
    src.sigma_r = 1e-4; src.r_trunc = 3e-4; src.z_inj = 0.0;
    if (orc_define_source(s, &src) < 0) return 5;
    if (orc_step(s, 60)) return 6;
    int64_t n = orc_num_packs(s);
    orc_packs pk;
    memset(&pk, 0, sizeof(pk));
    pk.n = n;
    pk.x = malloc(8 * n); pk.y = malloc(8 * n); pk.z = malloc(8 * n); pk.vx = malloc(8 * n); pk.vy = malloc(8 * n);
    pk.vz = malloc(8 * n); pk.e_int = malloc(8 * n); pk.h = malloc(8 * n); pk.w = malloc(8 * n);
    pk.id = malloc(8 * n); pk.q = malloc(8 * n); pk.tag = malloc(4 * n); pk.status = malloc(4 * n);
    if (orc_read_packs(s, &pk)) return 7;
    int64_t ne = orc_read_exits(s, NULL, 0), ns = orc_read_samples(s, NULL, 0);
    orc_exit *ex = malloc(sizeof(orc_exit) * (ne ? ne : 1));
    orc_sample *sm = malloc(sizeof(orc_sample) * (ns ? ns : 1));
    orc_read_exits(s, ex, ne);
    orc_read_samples(s, sm, ns);
    printf("OK packs %lld exits %lld samples %lld t %.3e\n", (long long)n, (long long)ne, (long long)ns,
           orc_current_time(s));
    free(ex); free(sm);
    void *bufs[] = {pk.x, pk.y, pk.z, pk.vx, pk.vy, pk.vz, pk.e_int, pk.h, pk.w, pk.id, pk.q, pk.tag, pk.status};
    for (size_t k = 0; k < sizeof(bufs) / sizeof(bufs[0]); ++k) free(bufs[k]);
    orc_destroy(s);
    free(phi); free(rf); free(uz); free(p); free(t); free(mask);
    return n > 0 && ns > 0 ? 0 : 8;
}
'''


def test_oracle_run_is_clean_under_sanitizers(tmp_path):
    odir = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I" + odir, str(src), os.path.join(odir, "mc_oracle.c"),
                    "-o", str(exe), "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK"), r.stdout + r.stderr
