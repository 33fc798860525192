"""Static checks of the HIP sources (CPU; needs hipcc, which cross-compiles).

Every device source must compile for gfx950 with a deleted min/max overload
for two different integral types (tests/mixed_minmax_guard.h): HIP's math
headers would otherwise evaluate such a call in double precision, in vector
registers, which once put the byte counts of the wide BF16 regeneration's
buffer descriptors into VGPRs and wrapped each staging load in a
readfirstlane loop.  A test that the guard itself works plants a mixed call
in a scratch source.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1409_0940_amd", "csrc")
GUARD = os.path.join(ROOT, "tests", "mixed_minmax_guard.h")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC),
                                reason="hipcc not available")


def _syntax_check(path, extra_includes=()):
    cmd = [HIPCC, "--offload-arch=gfx950", "-std=c++17", "--cuda-device-only", "-fsyntax-only",
           "-x", "hip", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
           *[f"-I{d}" for d in extra_includes], "-include", GUARD, path]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    return r.returncode, r.stderr


@pytest.mark.parametrize("src", sorted(f for f in os.listdir(CSRC) if f.endswith(".hip")))
def test_no_mixed_integer_min_max(src):
    rc, err = _syntax_check(os.path.join(CSRC, src))
    assert rc == 0, "\n".join(l for l in err.splitlines() if "error" in l)[:4000]


def test_guard_catches_a_mixed_call(tmp_path):
    src = tmp_path / "planted.hip"
    src.write_text("#include <hip/hip_runtime.h>\n#include <stdint.h>\n"
                   "__global__ void k(int64_t* p, int64_t n) { p[0] = min(n, 256); }\n")
    rc, err = _syntax_check(str(src))
    assert rc != 0 and "ambiguous" in err
