"""Host build and runner of the nested-step kernels under the HIP emulation.

The device code of ``nested.hip`` is compiled with g++ against the emulated
HIP runtime in this directory (``hip/hip_runtime.h``), by default with
AddressSanitizer, and run on one job whose outer Ritz matrix H_k is given as
its diagonal, sub- and super-diagonal.  Used by the CPU tests to check the
kernels' arithmetic and memory accesses without a GPU.
"""
from __future__ import annotations

import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "nested_driver.cpp")

# layout constants of the library (nks_internal.h, nks.h)
SC_COUNT, SC_ALPHA, SC_BETA, SC_GAMMA, SC_SV, SC_SW, SC_VN, SC_WN = 7, 0, 1, 2, 3, 4, 5, 6
ST_COUNT, RP_COUNT = 24, 16
ST_KUSED, ST_STATUS, ST_ELL, ST_RHI = 1, 2, 4, 5
RP_BNORM, RP_P, RP_ZMIN, RP_ZMAX, RP_INNER_DELTA = 0, 1, 2, 3, 4
NFEAT, LABEL_NK, LABEL_NELL, LABEL_DK = 16, 60, 4, 20
LABEL_WORDS = NFEAT + LABEL_NK * (1 + LABEL_NELL)
NEST_FINAL, NEST_LABEL = 0, 3
POLICY_FIXED, POLICY_DOUBLING = 0, 1


def build(out_dir: str, asan: bool = True, tsan: bool = False) -> str:
    """asan: AddressSanitizer (every access checked against its allocation);
    tsan: ThreadSanitizer instead (accesses of two threads to one location
    with no barrier between them); neither: plain -O2."""
    tag = "_tsan" if tsan else ("_asan" if asan else "")
    exe = os.path.join(out_dir, "nested_sim" + tag)
    cmd = ["g++", "-std=c++17", "-g", "-fno-omit-frame-pointer", "-I", HERE, "-I", os.path.join(ROOT, "include"),
           "-x", "c++", SRC, "-lpthread", "-o", exe]
    cmd[1:1] = ["-O1", "-fsanitize=thread"] if tsan else (["-O1", "-fsanitize=address"] if asan else ["-O2"])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return exe


def run(exe: str, alpha, beta, gamma, hermitian: bool, ell: int, *, vnorm=None, p: float = 0.0,
        mode: int = NEST_FINAL, label_points=(0, 0), tol: float = 1e-8, ell_policy: int = POLICY_FIXED,
        max_rhi: int = 50, rhi_tol: float = 1e-14, V: int = 256, mu: float = 0.0, timeout: float = 3600,
        label_head: bool = True, c_ref=None, fill: int = 0):
    """Runs one job; returns dict(status, report, c, label).  c = sgn(H_k) e_1
    as the kernel computes it (omega with |b| = 1 and unit scale factors).
    Label mode: label_head=False skips the launch that computes the features
    and the reference coefficients, which then come from c_ref.  fill: a
    byte (1..255) written over the scratch buffers before the launch (0: zeros)."""
    alpha = np.asarray(alpha, dtype=np.complex128)
    k = alpha.size
    sc = np.zeros((SC_COUNT, k + 2), dtype=np.complex128)
    sc[SC_ALPHA, 1:k + 1] = alpha
    sc[SC_BETA, 1:k] = np.asarray(beta, dtype=np.complex128)
    sc[SC_GAMMA, 1:k] = np.asarray(gamma, dtype=np.complex128)
    sc[SC_SV, 1:k + 1] = 1.0
    sc[SC_SW, 1:k + 1] = 1.0
    sc[SC_VN, 1:k + 1] = 1.0 if vnorm is None else np.asarray(vnorm, dtype=np.float64)
    sc[SC_WN, 1:k + 1] = 1.0
    hdr = np.zeros(16, dtype=np.int32)
    hdr[:14] = [k, ell, 0 if hermitian else 1, k, max_rhi, mode, label_points[0], label_points[1], V,
                POLICY_FIXED, ell_policy, 1, 0 if label_head else 1, fill]
    par = np.zeros(8, dtype=np.float64)
    par[:5] = [p, tol, rhi_tol, mu, 1.0]
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in.bin"), os.path.join(td, "out.bin")
        with open(fin, "wb") as f:
            f.write(hdr.tobytes() + par.tobytes() + np.zeros(8, np.int32).tobytes() +
                    np.zeros(8, np.float64).tobytes() + sc.tobytes())
            if mode == NEST_LABEL and not label_head:
                ref = np.zeros(k, np.complex128) if c_ref is None else np.asarray(c_ref, np.complex128)
                f.write(ref.tobytes())
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
                   TSAN_OPTIONS="halt_on_error=1:report_signal_unsafe=0")
        r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=timeout, env=env)
        if r.returncode != 0:
            raise RuntimeError(f"nested_sim failed ({r.returncode}):\n{r.stderr[-4000:]}")
        raw = open(fout, "rb").read()
    o = 0
    st = np.frombuffer(raw, np.int32, ST_COUNT, o); o += 4 * ST_COUNT
    rp = np.frombuffer(raw, np.float64, RP_COUNT, o); o += 8 * RP_COUNT
    om = np.frombuffer(raw, np.complex128, k, o); o += 16 * k
    lab = np.frombuffer(raw, np.float64, LABEL_WORDS, o) if mode == NEST_LABEL else None
    return dict(status=st.copy(), report=rp.copy(), c=om.copy(), label=None if lab is None else lab.copy(),
                log=r.stderr)
