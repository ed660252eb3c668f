"""The shared decision arithmetic of the pair-list builds (csrc/screen_math.h)
on the host: its exponential against the C library's over the screening
range, the screening bound against its closed form, the radius bands
against their log-uniform definition.  Compiled with g++ here; the device
build runs the same header (its records are compared with the host
packer's bit for bit in the GPU tests)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1011_4687_amd", "csrc")

PROG = r"""
#include <cmath>
#include <cstdio>
#include "screen_math.h"
using namespace envpot::sm;
int main() {
    // exp_neg over (-708, 0] (0 at -708 and below, by design): relative
    // error against the C library
    double worst = 0.0;
    for (int i = 0; i < 2000000; ++i) {
        const double x = -708.0 * i / 2000000.0;
        const double a = exp_neg(x), b = std::exp(x);
        const double r = std::fabs(a - b) / b;
        if (r > worst) worst = r;
    }
    std::printf("exp_rel %.3e\n", worst);
    std::printf("exp_edges %.17g %.17g %.17g\n", exp_neg(0.0), exp_neg(-708.5), exp_neg(1.0));
    // screening bound against its closed form at a few pairs
    const double ca = 0.7, cb = -0.3, a = 1.7, b = 0.45;
    const double n0a = std::pow(2 * a / kPi, 0.75), n0b = std::pow(2 * b / kPi, 0.75);
    double w2 = 0.0;
    for (int k = 0; k < 50; ++k) {
        const double r2 = 0.5 * k;
        const double ref = std::fabs(ca * cb) * n0a * n0b * std::pow(kPi / (a + b), 1.5) * std::exp(-a * b / (a + b) * r2);
        const double v = screen_bound(ca, cb, n0a, n0b, a, b, r2);
        const double r = std::fabs(v - ref) / ref;
        if (r > w2) w2 = r;
    }
    std::printf("bound_rel %.3e\n", w2);
    // radius bands: edges log-uniform between vmin and vmax (4 bands)
    const double vmin = 0.37, vmax = 1.9e3;
    const double lo = std::log(vmin), w = (std::log(vmax) - lo) / 4;
    double E[8] = {0, std::exp(lo + w), std::exp(lo + 2 * w), std::exp(lo + 3 * w), 0, 0, 0, 0};
    int bad = 0, prev = 0;
    for (int i = 0; i <= 100000; ++i) {
        const double v = vmin * std::pow(vmax / vmin, i / 100000.0);
        const int bnd = band_of(v, E, 4);
        const double t = (std::log(v) - lo) / w;
        const int ref = t < 1 ? 0 : t < 2 ? 1 : t < 3 ? 2 : 3;
        if (bnd != ref && std::fabs(t - std::round(t)) > 1e-12) ++bad;
        if (bnd < prev) ++bad;
        prev = bnd;
    }
    std::printf("band_bad %d\n", bad);
    return 0;
}
"""


@pytest.fixture(scope="module")
def out(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("sm")
    src = d / "t.cpp"
    src.write_text(PROG)
    exe = d / "t"
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off", "-Wno-unknown-pragmas", "-I", CSRC,
                    str(src), "-o", str(exe)], check=True)
    txt = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {ln.split()[0]: ln.split()[1:] for ln in txt.splitlines()}


def test_exponential_within_a_few_ulp(out):
    assert float(out["exp_rel"][0]) < 1e-15
    one, below, above = map(float, out["exp_edges"])
    assert one == 1.0 and below == 0.0 and above == 1.0  # clamped to the screening range


def test_screen_bound_closed_form(out):
    assert float(out["bound_rel"][0]) < 1e-14


def test_radius_bands_log_uniform_and_monotone(out):
    assert int(out["band_bad"][0]) == 0
