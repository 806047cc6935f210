"""The C-ABI library loads on the CPU host and exports every function include/gllmg.h declares;
host-side argument checking is exercised without touching a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gllmg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gllmg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_1402_5938_amd import gllmg
    lib = gllmg.lib()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(gllmg.EXPORTS)


def test_plan_and_validation_on_host():
    from paper_1402_5938_amd import gllmg
    cfg = gllmg.make_config(3, (16, 16, 16), 8, "p")
    nl, nbytes = gllmg.plan(cfg)
    assert nl == 7
    # G in FP64 dominates: 6 words per GLL point of the finest level
    assert nbytes > 6 * 8 * 4096 * 729
    cfg2 = gllmg.make_config(2, (4, 4), 4, "h")
    assert gllmg.plan(cfg2)[0] == 3
    bad = gllmg.make_config(3, (2, 2, 2), 17, "p")
    with pytest.raises(gllmg.GllmgError) as e:
        gllmg.plan(bad)
    assert e.value.status == gllmg.EINVAL
    bad = gllmg.make_config(4, (2, 2, 2), 4, "p")
    with pytest.raises(gllmg.GllmgError):
        gllmg.plan(bad)
    bad = gllmg.make_config(3, (1, 1, 1), 1, "p")       # no interior node
    with pytest.raises(gllmg.GllmgError):
        gllmg.plan(bad)
    # literal reading of the 16^3 p=8 hierarchy: stop at p = 1 on 16^3 (3375 coarse unknowns)
    assert gllmg.plan(gllmg.make_config(3, (16,) * 3, 8, "p", max_levels=4))[0] == 4
    # a single level beyond the dense-solve limit is allowed (products and smoothing only)
    assert gllmg.plan(gllmg.make_config(3, (16,) * 3, 8, "p", max_levels=1))[0] == 1
    for bad_k in (-1, 4097):
        with pytest.raises(gllmg.GllmgError) as e:
            gllmg.plan(gllmg.make_config(3, (4,) * 3, 4, "p", coarse_unknowns=bad_k))
        assert e.value.status == gllmg.EINVAL


@pytest.mark.parametrize("dim,ne,p,hier,k,ml", [
    (3, (16, 16, 16), 8, "p", 4096, 0), (3, (16, 16, 16), 8, "p", 3374, 0), (3, (16, 16, 16), 8, "p", 26, 0),
    (3, (8, 8, 8), 16, "p", 4096, 0), (3, (4, 4, 4), 16, "p", 4096, 0), (3, (4, 4, 4), 16, "p", 4096, 3),
    (2, (64, 64), 16, "p", 4096, 0), (2, (16, 16), 4, "h", 4096, 0), (2, (66, 66), 1, "h", 4096, 0),
    (3, (2, 2, 2), 4, "low", 4096, 0), (3, (4, 4, 2), 6, "low", 100, 0), (2, (24, 40), 3, "p", 50, 0),
])
def test_plan_matches_oracle_with_coarse_limit(dim, ne, p, hier, k, ml):
    """The library's level count equals the oracle's plan under the coarse-unknowns rule."""
    from paper_1402_5938_amd import gllmg
    from oracle import mg
    n = gllmg.plan(gllmg.make_config(dim, ne, p, hier, coarse_unknowns=k, max_levels=ml))[0]
    assert n == len(mg.plan_levels(dim, ne, p, hier, max_levels=ml, coarse_unknowns=k))


def test_null_arguments_rejected():
    from paper_1402_5938_amd import gllmg
    lib = gllmg.lib()
    assert lib.gllmg_plan(None, None, None) == gllmg.EINVAL
    assert b"NULL" in lib.gllmg_last_error()
    assert lib.gllmg_apply(None, 0, 0, 0, None, None, None) == gllmg.EINVAL
    assert lib.gllmg_destroy(None) == gllmg.OK


def test_binding_shares_torchs_hip_runtime():
    """The binding loads the library after torch, so the process maps a single HIP runtime
    (torch's device pointers and streams are only valid in the runtime that made them)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r); from paper_1402_5938_amd import gllmg; gllmg.lib(); "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"


def _function_bodies(src):
    """(name, body) of every top-level function definition in a C++ source (brace matching)."""
    out = []
    for m in re.finditer(r"\n(?:[A-Za-z_][\w:<>,*& ]*\s+)?([A-Za-z_]\w*)\s*\([^;{)]*(?:\)[^;{]*)?\)\s*(?:const\s*)?\{", src):
        depth, i = 1, m.end()
        while depth and i < len(src):
            depth += {"{": 1, "}": -1}.get(src[i], 0)
            i += 1
        out.append((m.group(1), src[m.end():i]))
    return out


def test_no_allocation_after_setup():
    """Device memory is allocated only by gllmg_setup; pinned memory, streams and events only by
    the host-resource pool's take_host_res, which only gllmg_setup calls (gllmg_destroy gives
    them back to the pool); the V-cycle graph is instantiated only by the capture helper
    (called at setup, by gllmg_set_lmax and by gllmg_set_graphs). So gllmg_plan's footprint is
    exact and a batch allocates nothing."""
    csrc = os.path.join(ROOT, "paper_1402_5938_amd", "csrc")
    allowed = {"hipMalloc": {"gllmg_setup"}, "hipHostMalloc": {"take_host_res"},
               "hipExtMallocWithFlags": set(), "hipMallocAsync": set(), "hipMallocManaged": set(),
               "hipStreamCreateWithFlags": {"take_host_res"}, "hipStreamCreate": set(),
               "hipEventCreateWithFlags": {"take_host_res"}, "hipEventCreate": set(),
               "hipGraphInstantiate": {"capture_vcycle"}, "take_host_res": {"gllmg_setup"}}
    found = {}
    for fn in sorted(os.listdir(csrc)):
        if not fn.endswith((".hip", ".h")):
            continue
        src = open(os.path.join(csrc, fn)).read()
        src = re.sub(r"//[^\n]*", "", src)
        for call in allowed:
            for m in re.finditer(r"\b%s\s*\(" % call, src):
                # the innermost enclosing function: the last definition starting before m
                owner = None
                for name, body in _function_bodies(src):
                    start = src.find(body)
                    if start <= m.start() < start + len(body):
                        owner = name
                if owner is None and re.match(r"%s\s*\([^;{]*\)\s*\{" % call, src[m.start():]):
                    continue  # the function's own definition
                found.setdefault(call, set()).add(owner)
    for call, owners in found.items():
        assert owners <= allowed[call], (call, owners)
    assert found.get("hipMalloc") == {"gllmg_setup"}
