"""Host-side AddressSanitizer run of the library's host code (CPU only).

Builds libvie_asan.so (host code instrumented, device code not; about two
minutes) and, in a child process with the ASan runtime preloaded, drives the
entry points that run on the host without a GPU: the two-photon
observables, the self-term coefficients, argument validation and the
failure paths of context and rooftop setup (which tear down what they built
when the device is missing).  Any ASan report fails the child.  Opt-in
(VIE_ASAN_TEST=1) because of the build time.
"""

import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import numpy as np
    from paper_2508_16471_amd import vie as V
    L = V.lib()
    assert V.LIB_PATH.endswith("libvie_asan.so"), V.LIB_PATH
    rng = np.random.default_rng(0)
    for _ in range(200):
        T = rng.standard_normal(4) + 1j * rng.standard_normal(4)
        V.hom_g2(T, 1.2, np.linspace(-3, 3, 17), V.VIE_NORM_R2, omega=(2.0, 1.0))
        V.hom_classical_p2(T)
    V.hom_g2(np.zeros(4, complex), 1.0, np.zeros(3))  # dark detector: NaN, VIE_OK
    for bad in ([np.nan, 0, 0, 0], [1, 1, 1, 1]):
        try:
            V.hom_g2(np.asarray(bad, complex), -1.0, np.zeros(2))
        except V.VieError:
            pass
    for kind in (0, 1):
        V.vie_self_term(kind, 2 * np.pi, 0.05)
    for code in range(-7, 1):
        V.strerror(code)
    assert V.vie_cnn_num_params() > 0
    # validation and failure paths of setup
    eps = np.full((3, 4, 5), 2.0)
    for args in [((eps * 0.5, 0.1, (0, 0, 0)),), ((eps, -1.0, (0, 0, 0)),),
                 ((np.full((2, 2, 300), 2.0), 0.1, (0, 0, 0)),), ((eps, 0.1, (0, 0, 0)),)]:
        try:
            V.vie_destroy(V.vie_setup(list(args), V.make_options(2 * np.pi)))
        except V.VieError:
            pass
    for e, h in ((eps * 0.5, 0.1), (np.full((2, 2, 200), 2.0), 0.1), (eps, 0.1)):
        try:
            V.vie_rt_destroy(V.vie_rt_setup(e, h, (0, 0, 0), 2 * np.pi))
        except V.VieError:
            pass
    L.vie_destroy(None)
    L.vie_rt_destroy(None)
    print("asan child ok")
""")


@pytest.mark.skipif(os.environ.get("VIE_ASAN_TEST") != "1", reason="opt-in: VIE_ASAN_TEST=1")
def test_host_code_under_asan():
    sys.path.insert(0, ROOT)
    from paper_2508_16471_amd import build_lib

    lib = build_lib.build(asan=True)
    rt = subprocess.run(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True, check=True).stdout.strip()
    env = dict(os.environ, VIE_LIB=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               PYTHONPATH=ROOT)
    p = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True,
                       timeout=600)
    assert p.returncode == 0 and "asan child ok" in p.stdout, p.stdout[-2000:] + p.stderr[-4000:]
