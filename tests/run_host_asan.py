"""Host code under AddressSanitizer, on the CPU (no GPU is touched).

Builds the library with AddressSanitizer on its host code
(`paper_1801_01037_amd/build.py --host-asan`), then, in a child process with
the sanitizer runtime preloaded, plans circuits of 4 to 33 qubits through the
C ABI: layered, QFT and mixed circuits with several-control gates, both
precisions, relabelled and standard storage, dense 5-qubit block plans, and
the code generation and hipRTC compilation of compiled passes. Any invalid
host memory access aborts the child. Run: python tests/run_host_asan.py
(a few minutes; not part of the pytest suites)."""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, __ROOT__)
import paper_1801_01037_amd as sv
sv.LIB_PATH = __LIB__
import qcircuits as qc
from tests.test_plan import mixed_circuit
count = 0
for n in (4, 5, 7, 9, 12, 13, 16, 20, 26, 30, 33):
    for dt in (sv.SV_C128, sv.SV_C64):
        for f in (sv.SV_FUSE, sv.SV_FUSE | sv.SV_NO_RELABEL):
            for g in (qc.layer_circuit(n, 8, n), qc.qft_circuit(n), mixed_circuit(n, 150, n + 1, mcu=True)):
                sv.sv_plan_inspect(n, dt, g, f)
                count += 1
        if n >= 5:
            sv.sv_plan_dense_inspect(n, qc.layer_circuit(n, 4, 2))
for dt in (sv.SV_C128, sv.SV_C64):
    sv.sv_plan_jit_check(14, dt, mixed_circuit(14, 80, 3, mcu=True))
    sv.sv_plan_jit_check(30, dt, qc.qft_circuit(30))
print("host code clean under AddressSanitizer:", count, "plans")
"""


def main() -> int:
    sys.path.insert(0, os.path.join(ROOT, "paper_1801_01037_amd"))
    import build as b
    lib = b.build(host_asan=True)
    rt = sorted(glob.glob(os.path.join(b.ROCM, "llvm", "lib", "clang", "*", "lib", "linux",
                                       "libclang_rt.asan-x86_64.so")))
    if not rt:
        print("AddressSanitizer runtime not found")
        return 2
    env = dict(os.environ, LD_PRELOAD=rt[-1], ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    code = CHILD.replace("__ROOT__", repr(ROOT)).replace("__LIB__", repr(lib))
    return subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    sys.exit(main())
