import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")


@pytest.fixture(scope="session")
def pdf_table():
    import workloads
    return workloads.synthetic_pdf()


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build()
    return oracle


# Independent Philox4x32-10: PyTorch's header-only engine, compiled as a test-only
# reference.  run([(seed, offset, subsequence)]) -> the four words of the block
# with counter (offset_lo, offset_hi, subsequence_lo, subsequence_hi), key = seed.
REF_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cinttypes>
int main() {
  unsigned long long seed, ev, sub;
  while (std::scanf("%llu %llu %llu", &seed, &ev, &sub) == 3) {
    at::Philox4_32 eng(seed, sub, ev);   /* counter = (ev_lo, ev_hi, sub_lo, sub_hi) */
    uint32_t a = eng(), b = eng(), c = eng(), d = eng();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
}
"""


@pytest.fixture(scope="session")
def torch_philox(tmp_path_factory):
    try:
        import torch
        TORCH_INC = os.path.join(os.path.dirname(torch.__file__), "include")
    except Exception:  # pragma: no cover
        TORCH_INC = None
    if TORCH_INC is None or not os.path.exists(os.path.join(TORCH_INC, "ATen/core/PhiloxRNGEngine.h")):
        pytest.skip("PyTorch Philox header not available")
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("philox")
    src = d / "ref.cpp"
    src.write_text(REF_SRC)
    exe = d / "ref"
    subprocess.run(["g++", "-std=c++17", "-O1", f"-I{TORCH_INC}", str(src), "-o", str(exe)],
                   check=True, capture_output=True)

    def run(triples):
        inp = "\n".join(f"{s} {e} {b}" for s, e, b in triples) + "\n"
        out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
        return [list(map(int, l.split())) for l in out.stdout.strip().splitlines()]
    return run
