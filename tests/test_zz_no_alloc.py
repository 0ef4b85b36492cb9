"""The allocation-free A-apply, stk_apply_A_noalloc, through the C ABI: its
output equals stk_apply_A's (the same kernels, with the shared-node slots in
the library's fixed per-GPU scratch array instead of context memory) on two
calls in a row, the second with a smaller input; it leaves the device's free
memory unchanged; and a level whose slots exceed the array is refused."""
import pytest
import torch

import inputs
from paper_2506_04157_amd import StokesContext
from paper_2506_04157_amd._lib import STK_EINVAL, StokesError

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def _fields(sc):
    X1, _ = sc.coords(which=1)
    T = inputs.SHField(2).temperature(X1)
    sc.set_fields(torch.tensor(inputs.viscosity_contrast(T, 1e4), device="cuda"))


def _compare(sc, level, dtype, seed):
    n2, _ = sc.sizes(level)
    x = torch.tensor(inputs.uniform(seed, 3 * n2), dtype=dtype, device="cuda")
    out = torch.full_like(x, float("nan"))
    free0 = torch.cuda.mem_get_info()[0]
    sc.apply_A_noalloc(x, out, level=level, bc=3)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    ref = sc.apply_A(x, level=level, bc=3)
    err = (torch.linalg.norm(out.double() - ref.double()) / torch.linalg.norm(ref.double())).item()
    print(f"level {level} {dtype}: rel. difference {err:.2e}, free memory change {free1 - free0} B", flush=True)
    assert torch.isfinite(out).all()
    assert err <= TOL[dtype]
    assert abs(free1 - free0) < (1 << 20)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_apply_matches_apply_A_on_two_calls(dtype):
    print(f"\n[no-alloc A-apply {dtype}]", flush=True)
    with StokesContext("shell", level=3, min_level=0, n_tan=2, n_rad=1) as sc:
        _fields(sc)
        _compare(sc, 3, dtype, 1)   # finest level: plane sweep with slots
        _compare(sc, 2, dtype, 2)   # then a smaller input on the same GPU scratch
        _compare(sc, 1, dtype, 3)   # element-parallel level: no slots


def test_noalloc_apply_refuses_a_level_beyond_the_scratch():
    print("\n[no-alloc refusal: shell 10x2 level 3]", flush=True)
    with StokesContext("shell", level=3, min_level=0, n_tan=10, n_rad=2) as sc:
        _fields(sc)
        n2, _ = sc.sizes()
        x = torch.zeros(3 * n2, dtype=torch.float64, device="cuda")
        y = torch.full_like(x, 7.0)
        # FP64 slots of 12,000 macros at level 3 exceed the 128 MiB array
        with pytest.raises(StokesError) as err:
            sc.apply_A_noalloc(x, y, bc=3)
        assert err.value.code == STK_EINVAL and "too large" in str(err.value)
        torch.cuda.synchronize()
        assert (y == 7.0).all()
        # the FP32 slots (half the bytes) fit
        _compare(sc, 3, torch.float32, 4)
