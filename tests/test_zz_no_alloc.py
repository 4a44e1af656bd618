"""The allocation-free entry point ttcf_pair_forces_static (device inputs and outputs, pair
lists in the library's static device scratch) against the allocating ttcf_debug_pair_form it
varies, which runs the same kernel: forces, W_xy, the Lees-Edwards offset and both flags are
equal bit for bit, on two calls in a row (the second with a smaller input, so that it runs
over what the first left in the scratch) and on a call whose capacity overflows."""
import sys

import numpy as np
import pytest

import ttcf_inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    from paper_2312_02990_amd import ttcf
    ttcf.lib()
    return ttcf


def run_static(T, sysd, r, gd, k, kcap=0):
    import torch
    n = sysd.n_atoms
    dev = torch.device("cuda:0")
    r_d = torch.from_numpy(np.ascontiguousarray(r, dtype=np.float64).ravel()).to(dev)
    f_d = torch.full((3 * n,), float("nan"), dtype=torch.float64, device=dev)
    out_d = torch.full((4,), float("nan"), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    code = T.ttcf_pair_forces_static(sysd, gd, k, 0.0, kcap, r_d.data_ptr(), f_d.data_ptr(),
                                     out_d.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    return code, f_d.cpu().numpy().reshape(3, n), out_d.cpu().numpy()


def check_same(T, s, seed, gd, k, kcap=0):
    r = I.perturbed_positions(s, seed, 0.08)
    sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
    say(f"static scratch: n={s.n} seed={seed} gamma_dot={gd} k={k} kcap={kcap}")
    ref = T.ttcf_debug_pair_form(sysd, r, gd, k, kcap=kcap)
    code, f, out = run_static(T, sysd, r, gd, k, kcap)
    assert code == T.TTCF_OK
    assert np.array_equal(f, ref["f"])
    assert out[0] == ref["w_xy"] and out[2] == ref["dxle"]
    assert bool(out[1]) == ref["close"] and bool(out[3]) == ref["overflow"]
    return ref


def test_static_scratch_matches_allocating_entry_point(T):
    k40 = int(round(0.4 / 0.0025))
    ref = check_same(T, I.System(8), 91, 1.0, k40)  # 2048 atoms, offset 0.4 L
    assert not ref["overflow"] and np.abs(ref["f"]).max() > 0.0
    check_same(T, I.System(4), 92, -1.0, 500)  # then 256 atoms over the same scratch


def test_static_scratch_reports_overflow_as_the_allocating_entry_point(T):
    ref = check_same(T, I.System(4), 93, 0.0, 0, kcap=1)
    assert ref["overflow"]

