"""mol_t_helmholtz_sweep_noalloc (the sweep for callers that cannot allocate)
gives the same results as mol_t_helmholtz_sweep, bit for bit, through the
C-ABI, on two calls in a row (the second smaller, reusing the static scratch
the first one filled), along both axes, in both precisions and for periodic and
Neumann lines."""
import sys

import pytest
import torch

from paper_1611_04214_amd import molt

pytestmark = pytest.mark.gpu


def _noalloc(g, axis, alpha, prec, x):
    out = torch.empty_like(x)
    batch = x.numel() // (g.nx * g.ny)
    rc = molt.mol_t_helmholtz_sweep_noalloc(g, axis, alpha, prec, x.data_ptr(), out.data_ptr(), batch,
                                            torch.cuda.current_stream().cuda_stream)
    assert rc == molt.MOLT_OK, molt.molt_last_error()
    return out


def _with_workspace(g, axis, alpha, prec, x):
    out = torch.empty_like(x)
    batch = x.numel() // (g.nx * g.ny)
    need = molt.molt_sweep_workspace_bytes(g, axis, prec, batch)
    work = molt.workspace(need)
    rc = molt.mol_t_helmholtz_sweep(g, axis, alpha, prec, x.data_ptr(), out.data_ptr(), batch, work.data_ptr(),
                                    work.numel(), torch.cuda.current_stream().cuda_stream)
    assert rc == molt.MOLT_OK, molt.molt_last_error()
    return out


@pytest.mark.parametrize("prec", [molt.MOLT_F64, molt.MOLT_F32])
@pytest.mark.parametrize("bc", [molt.MOLT_BC_PERIODIC, molt.MOLT_BC_NEUMANN])
@pytest.mark.parametrize("axis", [0, 1])
def test_noalloc_sweep_matches_the_workspace_sweep(prec, bc, axis):
    dt = torch.float64 if prec == molt.MOLT_F64 else torch.float32
    gen = torch.Generator().manual_seed(1611 + 4 * axis + 2 * bc + prec)
    # first call: 3 stacked 530 x 301 fields (several tiles, ragged tails);
    # second call: one 97 x 75 field on the scratch the first call left behind
    for (ny, nx, batch, alpha) in ((530, 301, 3, 41.0), (97, 75, 1, 7.5)):
        print(f"noalloc: axis={axis} bc={bc} prec={prec} shape=({batch},{ny},{nx})", flush=True)
        g = molt.make_grid(nx, ny, 0.0, 1.0, 0.0, 1.3, bc, 4)
        x = torch.rand(batch, ny, nx, generator=gen, dtype=torch.float64).to(dt).cuda()
        a = _noalloc(g, axis, alpha, prec, x)
        b = _with_workspace(g, axis, alpha, prec, x)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (a - b).abs().max().item()


def test_noalloc_full_size_field_and_repeat():
    """A 4096 x 4096 FP32 y sweep fits the static scratch; a second call on the
    same scratch with a smaller field still matches."""
    for n in (4096, 1000):
        print(f"noalloc: full-size shape=({n},{n})", flush=True)
        g = molt.make_grid(n, n, bc=molt.MOLT_BC_PERIODIC)
        x = torch.rand(n, n, generator=torch.Generator().manual_seed(n)).cuda()
        a = _noalloc(g, 1, 278.3, molt.MOLT_F32, x)
        b = _with_workspace(g, 1, 278.3, molt.MOLT_F32, x)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-q"]))
