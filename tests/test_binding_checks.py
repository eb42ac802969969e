"""The Python binding refuses tensors that do not match the call before it
hands an address to the library (a mismatched dtype or size would make the
kernels read or write outside the tensor).  CPU tensors suffice: every check
runs before the first library call that touches a device."""
import pytest
import torch

from paper_1611_04214_amd import molt


@pytest.fixture(scope="module")
def lib():
    return molt.load()


def _raises(fn, text):
    with pytest.raises(molt.MoltError) as e:
        fn()
    assert e.value.status == molt.MOLT_EINVAL
    assert text in str(e.value)


def test_step_and_solve_check_dtype_size_layout_and_device(lib):
    g = molt.make_grid(16, 12, bc=molt.MOLT_BC_PERIODIC)
    p64 = molt.make_params(0.05, 1e-3, precision=molt.MOLT_F64)
    p32 = molt.make_params(0.05, 1e-3, precision=molt.MOLT_F32)
    good64 = torch.zeros(12, 16, dtype=torch.float64)
    _raises(lambda: molt.step(good64.float(), g, p64), "float32")
    _raises(lambda: molt.step(good64, g, p32), "float64")
    _raises(lambda: molt.solve(torch.zeros(12, 15, dtype=torch.float64), g, p64, 1), "192")
    _raises(lambda: molt.solve(torch.zeros(16, 12, dtype=torch.float64).t(), g, p64, 1), "contiguous")
    _raises(lambda: molt.step(good64, g, p64), "HIP device")
    # the vector model's fields hold two components
    pv = molt.make_params(0.05, 1e-3, precision=molt.MOLT_F64, model=molt.MOLT_MODEL_VCH)
    _raises(lambda: molt.solve(good64, g, pv, 1), "384")
    # a BDF3 history holds two fields
    p3 = molt.make_params(0.05, 1e-3, precision=molt.MOLT_F64, stepper=molt.MOLT_BDF3, have_prev=2)
    _raises(lambda: molt.step(torch.zeros(12, 16, dtype=torch.float64), g, p3,
                              u_prev=torch.zeros(12, 16, dtype=torch.float64)), "384")


def test_sweep_checks_its_field_and_output(lib):
    g = molt.make_grid(16, 8)
    _raises(lambda: molt.sweep(torch.zeros(8, 16, dtype=torch.float16), g, 0, 10.0), "float16")
    _raises(lambda: molt.sweep(torch.zeros(8, 15), g, 0, 10.0), "multiple of 128")
    _raises(lambda: molt.sweep(torch.zeros(3, 8, 16), g, 0, 10.0, out=torch.zeros(2, 8, 16)), "384")
    _raises(lambda: molt.sweep(torch.zeros(8, 16), g, 0, 10.0, out=torch.zeros(8, 16, dtype=torch.float64)),
            "float64")


def test_batch_checks_every_instance(lib):
    g = molt.make_grid(16, 16)
    p = molt.make_params(0.05, 1e-3, precision=molt.MOLT_F32)
    specs = [(g, p, torch.zeros(16, 16), 2), (g, p, torch.zeros(16, 15), 2)]
    _raises(lambda: molt.solve_batch(specs), "instance 1")
    _raises(lambda: molt.solve_batch(specs[:1]), "instance 0's field must be on a HIP device")
    _raises(lambda: molt.solve_batch([]), "no instances")
