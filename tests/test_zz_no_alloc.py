"""gllmg_apply_noalloc (the product with the library's static element-vector buffer) against
gllmg_apply, through the C ABI: bit for bit on two calls in a row (the second on a smaller
level and then on a smaller problem), FP64 and FP32, Dirichlet and Neumann, against the oracle
to the FP64 bar, and a level too large for the static buffer rejected before anything runs."""

import ctypes

import numpy as np
import pytest

from gpu_helpers import build_pair, fp64_close, random_vec, to_dev, to_np

pytestmark = pytest.mark.gpu


def _noalloc(G, x, y, level, prec, neumann=0):
    from paper_1402_5938_amd import gllmg
    import torch
    s = torch.cuda.current_stream().cuda_stream
    return gllmg.lib().gllmg_apply_noalloc(G.h, level, prec, neumann, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(s))


def _free_bytes():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_noalloc_product_equals_apply_two_calls_in_a_row():
    import torch
    from paper_1402_5938_amd import gllmg
    # 3D warped, variable coefficient: level 0 at p = 8 (3 x 2 x 2 elements), level 1 at p = 4
    G, H = build_pair(3, (3, 2, 2), 8, max_levels=2)
    sizes = []
    for level, prec in [(0, gllmg.F64), (1, gllmg.F64)]:
        lv = H.levels[level]
        x = to_dev(random_vec(lv.mesh.N, 5 + level))
        for neumann in (0, 1):
            ref = G.apply(x, l=level, neumann=bool(neumann))
            y = torch.full_like(x, float("nan"))
            assert _noalloc(G, x, y, level, prec, neumann) == gllmg.OK, gllmg.lib().gllmg_last_error()
            torch.cuda.synchronize()
            assert torch.equal(y, ref)
            ok, e = fp64_close(to_np(y), lv.op.apply(to_np(x), neumann=bool(neumann)))
            assert ok, e
        sizes.append(lv.mesh.N)
    assert sizes[1] < sizes[0]
    # no device memory is taken by further calls
    x0 = to_dev(random_vec(H.levels[0].mesh.N, 9))
    y0 = torch.empty_like(x0)
    free0 = _free_bytes()
    for _ in range(3):
        assert _noalloc(G, x0, y0, 0, gllmg.F64) == gllmg.OK
    assert _free_bytes() == free0
    G.close()
    # then a smaller problem (2D, p = 4) on the same device: the array keeps the last call's
    # contents, which the next call overwrites before reading
    G2, H2 = build_pair(2, (3, 2), 4, max_levels=1)
    x2 = to_dev(random_vec(H2.levels[0].mesh.N, 3))
    y2 = torch.empty_like(x2)
    assert _noalloc(G2, x2, y2, 0, gllmg.F64) == gllmg.OK
    torch.cuda.synchronize()
    assert torch.equal(y2, G2.apply(x2))
    G2.close()


def test_noalloc_product_fp32():
    import torch
    from paper_1402_5938_amd import gllmg
    G, H = build_pair(3, (2, 2, 1), 12, max_levels=2, vcycle_prec="f32")
    for level in (0, 1):
        x = to_dev(random_vec(H.levels[level].mesh.N, 21 + level), torch.float32)
        y = torch.empty_like(x)
        assert _noalloc(G, x, y, level, gllmg.F32) == gllmg.OK
        torch.cuda.synchronize()
        assert torch.equal(y, G.apply(x, l=level))
    G.close()


def test_noalloc_rejects_a_level_beyond_the_static_buffer():
    import torch
    from paper_1402_5938_amd import gllmg, inputs
    # 24 x 24 x 12 hexes at p = 8: 6912 * 729 * 8 bytes = 40.3 MB of element vectors > 32 MiB
    cfg = gllmg.make_config(3, (24, 24, 12), 8, "p", max_levels=1)
    G = gllmg.Problem(cfg, inputs.map_identity(), inputs.field_const(1.0))
    x = torch.ones(G.nnodes(0), dtype=torch.float64, device="cuda")
    y = torch.full_like(x, 7.0)
    assert _noalloc(G, x, y, 0, gllmg.F64) == gllmg.EINVAL
    assert b"static scratch" in gllmg.lib().gllmg_last_error()
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())      # nothing was enqueued
    G.close()
