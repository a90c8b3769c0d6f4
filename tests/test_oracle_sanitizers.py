"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): a small C driver exercises every exported function of
oracle/ivr_oracle.h on a jittered quadratic block (reference render with each
field and both clip planes, the method mode with every interior method and the
pixel-accuracy record, the convergence studies, Hessian, fields, Delta P and
point location), built with -fsanitize=address,undefined and no recovery, so
that any out-of-bounds access, leak or undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include "ivr_oracle.h"

int main(void)
{
    /* degree 2, 4^3 control points on the unit cube, interior jittered */
    const double knots[7] = {0, 0, 0, 0.5, 1, 1, 1};
    const double g[4] = {0, 0.25, 0.75, 1};
    double cp[64 * 4], sc[64], disp[64 * 3];
    for (int k = 0; k < 4; ++k)
        for (int j = 0; j < 4; ++j)
            for (int i = 0; i < 4; ++i) {
                const int q = i + 4 * (j + 4 * k);
                const int inner = i > 0 && i < 3 && j > 0 && j < 3 && k > 0 && k < 3;
                cp[4 * q + 0] = g[i] + (inner ? 0.04 * sin(1.0 + q) : 0.0);
                cp[4 * q + 1] = g[j] + (inner ? 0.04 * cos(2.0 + q) : 0.0);
                cp[4 * q + 2] = g[k] + (inner ? 0.04 * sin(3.0 + q) : 0.0);
                cp[4 * q + 3] = 1.0 + 0.1 * ((i + j + k) % 2);
                sc[q] = 0.5 + 0.4 * sin(2.0 * g[i] + g[j] - g[k]);
                disp[3 * q + 0] = 0.01 * cp[4 * q + 1];
                disp[3 * q + 1] = 0.02 * cp[4 * q + 2];
                disp[3 * q + 2] = -0.01 * cp[4 * q + 0];
            }
    orc_patch P = {{2, 2, 2}, {4, 4, 4}, {knots, knots, knots}, cp, sc, 1, disp};
    orc_scene *s = orc_prepare(&P, 1, sqrt(3.0));
    if (!s) return 2;
    const double tx[4] = {0, 0.3, 0.7, 1}, trgba[16] = {0.1, 0.2, 0.9, 0.1, 0.9, 0.5, 0.1, 0.6,
                                                       0.3, 0.8, 0.4, 0.9, 0.7, 0.7, 0.2, 0.4};
    orc_tf tf = {4, tx, trgba, 4.0, {0.0, 1.0}};
    orc_camera cam = {{2.4, 1.9, 1.6}, {0.5, 0.5, 0.5}, {0, 0, 1}, 40.0, 12, 12};
    double rgba[144 * 4], depth[144], dp[144];
    int32_t bad[144];
    orc_pixel_diag diag[144];
    for (int field = 0; field < 3; ++field)
        for (int planes = 0; planes < 2; ++planes) {
            orc_opts o = {512.0, 1, 2, 1e-4, planes, {0.5, 0.5, 0.5}, {0.3, -0.2, 0.9}, planes ? 3.0 : 0.0, field};
            if (orc_render_pixels(s, &cam, &tf, &o, NULL, 144, rgba, depth, diag) != 0) return 3;
        }
    for (int m = 0; m <= 8; ++m) {
        orc_method_opts mo = {1e-5, 0.0, 1.0, 0.1, 0.025, 4, 1, 2, m};
        int64_t steps = 0;
        if (orc_render_pixels_method(s, &cam, &tf, &mo, NULL, 144, rgba, &steps, dp, bad) != 0) return 4;
    }
    for (int m = 1; m <= 7; ++m) {
        int32_t it;
        if (!(orc_table1_newton(m, 1.0 / 64, m == 7 ? 100.0 : 1.0, &it) >= 0.0)) return 5;
        const double a[3] = {0.1, 0.2, 0.15}, b[3] = {0.9, 0.75, 0.85};
        if (!(orc_path_error(&P, a, b, m, 1.0 / 32, 1.0, &it) >= 0.0)) return 6;
    }
    const double p[3] = {0.3, 0.6, 0.45};
    double x[3], J[9], H[27], v;
    if (orc_eval_hessian(&P, p, x, J, H) != 0) return 7;
    for (int field = 0; field < 3; ++field)
        if (orc_field(&P, p, field, &v) != 0) return 8;
    if (!(orc_delta_p(&cam, 77, x) >= 0.0)) return 9;
    double pts[6] = {0.5, 0.5, 0.5, 0.2, 0.3, 0.4}, pl[6];
    int32_t blk[2] = {-1, -2};
    orc_locate(s, pts, 2, blk, pl, NULL);
    orc_fragment fr[64];
    double o[3], d[3];
    orc_camera_ray(&cam, 6.5, 5.5, o, d);
    if (orc_ray_fragments(s, o, d, fr, 64) < 0) return 10;
    orc_free(s);
    printf("ok\n");
    return 0;
}
'''


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = [cc, "-std=c11", "-O1", "-g", "-D_GNU_SOURCE", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
           str(src), os.path.join(ROOT, "oracle", "ivr_oracle.c"), "-o", str(exe), "-lm", "-lpthread"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0 and res.stdout.strip() == "ok", (res.returncode, res.stdout[-2000:], res.stderr[-4000:])
