"""The host code of the library under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

api.cpp and bath.cpp are rebuilt with the sanitizers on the host side only
(each -fsanitize option behind -Xarch_host; device code is untouched) and
linked with the kernel objects of the regular build into a separate
library.  A small C++ driver then runs every host path that needs no GPU:
the bath discretisation over many sizes and kinds, and each argument check
of iesh_create and iesh_eigh_batched with iesh_last_error(NULL).  Any
sanitizer report fails the run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2212_00518_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2212_00518_amd", "_build")
KERNELS = ["k_eig", "k_prop", "k_hop", "k_lowdin", "k_compact", "k_adjoint", "k_jacobi",
           "eigh_noalloc", "k_dense"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

DRIVER = r'''
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#include "iesh.h"

static int fails = 0;
#define EXPECT(c) do { if (!(c)) { std::printf("FAILED %s:%d %s\n", __FILE__, __LINE__, #c); ++fails; } } while (0)

static iesh_model_desc model(std::vector<double>& e, std::vector<double>& w, int n_elec) {
  iesh_model_desc m;
  std::memset(&m, 0, sizeof m);
  m.kind = IESH_MODEL_HARMONIC;
  m.n_bath = (int)e.size();
  m.n_elec = n_elec;
  m.eps = e.data();
  m.w = w.data();
  m.mass = 2000.0;
  m.Gamma = 0.01;
  m.params[0] = 2e-4;
  m.params[1] = 20.0;
  m.params[2] = -3.8e-3;
  return m;
}

static iesh_run_desc run() {
  iesh_run_desc r;
  std::memset(&r, 0, sizeof r);
  r.n_traj = 4;
  r.precision = IESH_FP64;
  r.dt = 20.0;
  r.kT = 1e-3;
  return r;
}

int main() {
  int a, b, c;
  EXPECT(iesh_version(&a, &b, &c) == IESH_OK);
  // discretisation over sizes and kinds
  for (int kind = 0; kind < 3; ++kind)
    for (int M = 1; M <= 335; M += (M < 70 ? 1 : 37)) {
      std::vector<double> e(M), w(M);
      const int rc = iesh_discretize(kind, M, -0.05, 0.05, 0.0, e.data(), w.data());
      if (kind == 2 && (M % 2)) { EXPECT(rc == IESH_EINVAL); continue; }
      EXPECT(rc == IESH_OK);
      double s = 0.0;
      for (int k = 0; k < M; ++k) s += w[k];
      EXPECT(std::fabs(s - 0.1) < 1e-12);
    }
  EXPECT(iesh_discretize(0, 0, -0.05, 0.05, 0.0, nullptr, nullptr) == IESH_EINVAL);
  // bath of a workload: one and two leads, both placements, levels below mu
  for (int kind = 0; kind < 3; ++kind)
    for (int leads = 1; leads <= 2; ++leads)
      for (int M = 4; M <= 320; M += 4 * (M < 40 ? 1 : 19)) {
        iesh_bath_desc d;
        std::memset(&d, 0, sizeof d);
        d.kind = kind;
        d.M = M;
        d.n_leads = leads;
        d.placement = (M / 4) % 2;
        d.W = 0.1;
        d.mu = 0.01;
        std::vector<double> e(M), w(M);
        std::vector<int32_t> l(M);
        int32_t nb = -1;
        const int rc = iesh_bath(&d, e.data(), w.data(), l.data(), &nb);
        if (kind == 2 && (M / leads) % 2) { EXPECT(rc == IESH_EINVAL); continue; }
        EXPECT(rc == IESH_OK);
        EXPECT(nb >= 0 && nb <= M);
        double s = 0.0;
        for (int k = 0; k < M; ++k) s += w[k];
        EXPECT(std::fabs(s - 0.1) < 1e-12);
      }
  EXPECT(iesh_bath(nullptr, nullptr, nullptr, nullptr, nullptr) == IESH_EINVAL);
  // each argument check of iesh_create, before any device call
  std::vector<double> e(8), w(8, 0.1 / 8);
  for (int k = 0; k < 8; ++k) e[k] = -0.05 + k * 0.1 / 7;
  iesh_ctx* ctx = nullptr;
  {
    iesh_model_desc m = model(e, w, 4);
    iesh_run_desc r = run();
    r.dt = 0.0;
    EXPECT(iesh_create(&m, 1, nullptr, &r, nullptr, &ctx) == IESH_EINVAL && !ctx);
    EXPECT(std::strstr(iesh_last_error(nullptr), "dt") != nullptr);
  }
  {
    std::vector<double> e2 = e;
    e2[3] = 1.0;  // not ascending
    iesh_model_desc m = model(e2, w, 4);
    iesh_run_desc r = run();
    EXPECT(iesh_create(&m, 1, nullptr, &r, nullptr, &ctx) == IESH_EINVAL);
    EXPECT(std::strstr(iesh_last_error(nullptr), "ascending") != nullptr);
  }
  {
    iesh_model_desc m = model(e, w, 9);  // more electrons than bath levels
    iesh_run_desc r = run();
    EXPECT(iesh_create(&m, 1, nullptr, &r, nullptr, &ctx) == IESH_EINVAL);
  }
  {
    std::vector<int32_t> lead(8, 2);
    iesh_model_desc m = model(e, w, 4);
    m.lead = lead.data();
    iesh_run_desc r = run();
    EXPECT(iesh_create(&m, 1, nullptr, &r, nullptr, &ctx) == IESH_EINVAL);
  }
  {
    iesh_model_desc m = model(e, w, 4);
    iesh_run_desc r = run();
    r.bias = 0.01;  // no lead labels
    EXPECT(iesh_create(&m, 1, nullptr, &r, nullptr, &ctx) == IESH_EINVAL);
    r.bias = 0.0;
    r.dt_levels = 2;  // no threshold
    EXPECT(iesh_create(&m, 1, nullptr, &r, nullptr, &ctx) == IESH_EINVAL);
    r.dt_levels = 0;
    r.eig_max_iter = 500;
    EXPECT(iesh_create(&m, 1, nullptr, &r, nullptr, &ctx) == IESH_EINVAL);
    r.eig_max_iter = 0;
    std::vector<int32_t> tm(4, 3);  // model index out of range
    EXPECT(iesh_create(&m, 1, tm.data(), &r, nullptr, &ctx) == IESH_EINVAL);
  }
  EXPECT(iesh_create(nullptr, 1, nullptr, nullptr, nullptr, &ctx) == IESH_EINVAL);
  EXPECT(iesh_destroy(nullptr) == IESH_OK);
  // the dense eigen-solver's argument checks
  double H[4] = {1, 0, 0, 1}, lam[2], Q[4];
  EXPECT(iesh_eigh_batched(H, 0, 1, lam, Q, nullptr, IESH_MEM_HOST, nullptr) == IESH_EINVAL);
  EXPECT(iesh_eigh_batched(H, 337, 1, lam, Q, nullptr, IESH_MEM_HOST, nullptr) == IESH_EINVAL);
  EXPECT(iesh_eigh_batched(H, 2, -1, lam, Q, nullptr, IESH_MEM_HOST, nullptr) == IESH_EINVAL);
  EXPECT(iesh_eigh_batched(H, 2, 1, lam, Q, nullptr, 9, nullptr) == IESH_EINVAL);
  EXPECT(iesh_eigh_batched(nullptr, 2, 0, nullptr, nullptr, nullptr, IESH_MEM_HOST, nullptr) == IESH_OK);
  EXPECT(std::strlen(iesh_last_error(nullptr)) < 200);
  std::printf("host paths done, %d failures\n", fails);
  return fails ? 1 : 0;
}
'''


def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    objs = [os.path.join(BUILD, k + ".o") for k in KERNELS]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("kernel objects not built (run __graft_entry__.build())")
    inc = os.path.join(ROOT, "include")
    flags = ["-O1", "-g", "-fPIC", "-std=c++17", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    host = []
    for src in ("api.cpp", "bath.cpp"):
        o = str(tmp_path / (src + ".o"))
        subprocess.run([hipcc, "-x", "hip", *flags, *SAN, "-c", os.path.join(CSRC, src), "-o", o],
                       check=True, capture_output=True)
        host.append(o)
    lib = str(tmp_path / "libiesh_san.so")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *host, *objs, *SAN, "-o", lib],
                   check=True, capture_output=True)
    drv = tmp_path / "driver.cpp"
    drv.write_text(DRIVER)
    exe = str(tmp_path / "driver")
    dobj = str(tmp_path / "driver.o")
    subprocess.run([hipcc, "-x", "c++", "-O1", "-g", "-std=c++17", "-I", inc, *SAN, "-c", str(drv),
                    "-o", dobj], check=True, capture_output=True)
    subprocess.run([hipcc, *SAN, dobj, lib, "-Wl,-rpath," + str(tmp_path), "-o", exe], check=True,
                   capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "0 failures" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
