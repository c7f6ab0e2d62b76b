"""The library's device memory through l1ls_set_allocator.

The Python binding installs PyTorch's caching allocator, so every block the
library holds shows in torch.cuda.memory_allocated: an instance adds its
l1ls_instance_bytes at generation and gives them back at l1ls_free, and
solves leave nothing behind.  A counting allocator checks that every block
goes back to the allocator that made it.
"""
import ctypes

import pytest

torch = pytest.importorskip("torch")

import paper_1503_03520_amd as L  # noqa: E402

pytestmark = pytest.mark.gpu

# torch rounds every block up to a multiple of 512 bytes
ROUND = 512


def _allocated():
    torch.cuda.synchronize()
    return torch.cuda.memory_allocated()


def test_instance_memory_comes_from_torch_and_goes_back():
    L.lib()
    L.use_torch_allocator()
    before = _allocated()
    inst = L.l1ls_generate(1 << 16, 1 << 15, 1e3, 300, 1.0, 1503035401, rounds=2,
                           storage=L.STORE_F32 | L.STORE_F64 | L.STORE_BLK32)
    held = _allocated() - before
    nb = inst.nbytes()
    print(f"\n[case] instance bytes {nb}, torch allocated {held}", flush=True)
    # each block is rounded up by less than 512 bytes
    assert nb > 0 and nb <= held <= nb + 256 * ROUND
    x, rep, _ = L.l1ls_solve_fista(inst, max_iter=64, rel_gap_tol=0.0, precision=L.F32, polish=1)
    xn, rn, _ = L.l1ls_solve_cg_newton(inst, max_iter=2, rel_gap_tol=1e-12, precision=L.F64)
    del x, xn
    # solver workspaces and temporaries are all returned
    assert _allocated() - before == held
    inst.free()
    assert _allocated() == before


def test_blocks_go_back_to_the_allocator_that_made_them():
    lib = L.lib()
    live = {}
    counts = {"a": 0, "f": 0}

    def alloc(ctx, nbytes):
        p = torch.cuda.caching_allocator_alloc(int(nbytes))
        live[p] = int(nbytes)
        counts["a"] += 1
        return p

    def free(ctx, ptr, nbytes):
        assert live.pop(ptr) == int(nbytes)
        counts["f"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    fa, ff = L._ALLOC_FN(alloc), L._FREE_FN(free)
    spec = L.Allocator(fa, ff, None)
    try:
        assert lib.l1ls_set_allocator(ctypes.byref(spec)) == 0
        inst = L.l1ls_generate(4096, 2048, 1e2, 20, 1.0, 1503035402, rounds=2)
        made = counts["a"]
        assert made > 0 and len(live) == made - counts["f"]
        held = sum(live.values())
        assert held == inst.nbytes()
        # another allocator installed: the instance's blocks still go back here
        L.use_hip_malloc()
        x, rep, _ = L.l1ls_solve_fista(inst, max_iter=32, rel_gap_tol=0.0, precision=L.F64)
        assert counts["a"] == made
        inst.free()
        torch.cuda.synchronize()
        assert not live and counts["f"] == counts["a"]
    finally:
        L.use_torch_allocator()

