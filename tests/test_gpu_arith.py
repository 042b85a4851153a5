"""The short FP64 division and square root of the face code (div_nr and
sqrt_pos: the hardware estimates refined by one Newton-Raphson step plus a
residual correction, and the compiler's own square root steps without range
scaling) against the IEEE operations on the GPU, bit for bit on 4 M seeded
operands. The check program is built by __graft_entry__.build()."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_division_and_square_root_are_correctly_rounded():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    exe = os.path.join(HERE, "native", "arith_check")
    assert os.path.exists(exe), "tests/native/arith_check is missing: run __graft_entry__.build()"
    print("arith check: div_nr and sqrt_pos vs IEEE on 4 M operands", flush=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(out.stdout, flush=True)
    assert out.returncode == 0, out.stdout + out.stderr
    fields = dict(zip(out.stdout.split()[::2], out.stdout.split()[1::2]))
    assert fields["div_nr_mismatch"] == "0" and fields["sqrt_pos_mismatch"] == "0"
