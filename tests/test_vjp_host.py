"""Host check of the reverse-mode HLLD flux (csrc/hlld_vjp.h) against central
differences of the forward flux (csrc/mhd_dev.h, hlld_flux), both compiled
for the CPU with g++ through a minimal stand-in for the HIP runtime header.

For random left/right states and normal fields, in double precision, the
cotangents of all 15 inputs for a random cotangent of the 7 flux components
must equal the difference quotients of lam . F.  A quotient is compared only
where the flux is smooth at that input: the one-sided quotients on both
sides agree, so no wave-pattern or degenerate-state branch lies within the
step."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1705_10774_amd", "csrc")

SHIM = r"""
#pragma once
#include <cmath>
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
inline float __builtin_amdgcn_rcpf(float x) { return 1.0f / x; }
inline float __builtin_amdgcn_sqrtf(float x) { return std::sqrt(x); }
using std::fabs;
using std::sqrt;
"""

PROG = r"""
#include <cstdio>
#include <random>
#include "mhd_dev.h"
#include "hlld_vjp.h"
using namespace dsp;

static double phi(const double* x, const double* lam, double gamma) {
  double f[8];
  hlld_flux<double>(x, x + 7, x[14], gamma, f);
  double s = 0.0;
  for (int q = 0; q < 7; ++q) s += lam[q] * f[q];
  return s;
}

int main() {
  std::mt19937_64 rng(20170531);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  const double gamma = 5.0 / 3.0;
  long compared = 0, skipped = 0;
  double worst = 0.0;
  for (int it = 0; it < 4000; ++it) {
    double x[15], lam[7];
    const double sc = (it % 4 == 0) ? 3.0 : 0.5;  // some supersonic pairs
    for (int s = 0; s < 2; ++s) {
      double* w = x + 7 * s;
      w[0] = 0.5 + 0.75 * (U(rng) + 1.0);
      for (int m = 1; m < 4; ++m) w[m] = sc * U(rng);
      w[4] = 0.1 + (U(rng) + 1.0);
      w[5] = U(rng);
      w[6] = U(rng);
    }
    x[14] = U(rng);
    for (int q = 0; q < 7; ++q) lam[q] = U(rng);
    double g[15];
    hlld_vjp<double>(x, x + 7, x[14], gamma, lam, g, g + 7, g[14]);
    for (int j = 0; j < 15; ++j) {
      const double h = 1e-6 * (1.0 + std::fabs(x[j]));
      double xp[15], xm[15];
      for (int m = 0; m < 15; ++m) xp[m] = xm[m] = x[m];
      xp[j] += h;
      xm[j] -= h;
      const double f0 = phi(x, lam, gamma), fp = phi(xp, lam, gamma), fm = phi(xm, lam, gamma);
      const double dp = (fp - f0) / h, dm = (f0 - fm) / h, dc = (fp - fm) / (2.0 * h);
      const double scale = 1.0 + std::fabs(dc);
      if (std::fabs(dp - dm) > 1e-3 * scale) {  // a branch within the step
        ++skipped;
        continue;
      }
      ++compared;
      const double rel = std::fabs(g[j] - dc) / scale;
      if (rel > worst) worst = rel;
    }
  }
  std::printf("%ld %ld %.6e\n", compared, skipped, worst);
  return 0;
}
"""


def test_hlld_reverse_mode_matches_central_differences(tmp_path):
    (tmp_path / "hip").mkdir()
    (tmp_path / "hip" / "hip_runtime.h").write_text(SHIM)
    src = tmp_path / "vjp_check.cpp"
    src.write_text(PROG)
    exe = tmp_path / "vjp_check"
    subprocess.run(["g++", "-std=c++17", "-O2", "-I", str(tmp_path), "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    compared, skipped, worst = int(out[0]), int(out[1]), float(out[2])
    print("compared", compared, "skipped", skipped, "worst", worst)
    assert compared >= 0.95 * (compared + skipped)
    assert worst < 1e-6
