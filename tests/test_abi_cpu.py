"""CPU checks of the C-ABI library: it loads and exports every declared symbol."""
import ctypes
import os
import subprocess

from paper_0811_4331_amd import wdmg


def test_header_declares_the_boundary():
    syms = wdmg.header_symbols()
    for name in ("wdmg_create", "wdmg_destroy", "wdmg_set_gauge", "wdmg_set_mass", "wdmg_apply_D",
                 "wdmg_mg_setup", "wdmg_apply_Dc", "wdmg_restrict", "wdmg_prolong", "wdmg_smooth",
                 "wdmg_solve", "wdmg_solve_bicgstab", "wdmg_get_prolongator", "wdmg_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = wdmg.load()
    for name in wdmg.header_symbols():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", wdmg.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert set(wdmg.header_symbols()) <= exported


def test_default_params_are_the_papers_constants():
    lib = wdmg.load()
    p = wdmg.MgParams()
    lib.wdmg_default_mg_params(ctypes.byref(p))
    assert abs(p.omega - 0.8) < 1e-15 and p.nu_pre == 2 and p.nu_post == 2 and p.coarse_cycles == 4
    s = wdmg.SolveParams()
    lib.wdmg_default_solve_params(ctypes.byref(s))
    assert s.restart == 50 and s.tol == 1e-10


def test_create_rejects_bad_dims_without_a_gpu_call():
    lib = wdmg.load()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int * 4)(4, 4, 1, 4)
    assert lib.wdmg_create(ctypes.byref(h), dims, None, None) == -2
    assert lib.wdmg_create(None, dims, None, None) == -1


def test_struct_layouts_match_header_sizes():
    # the C structs as the compiler lays them out, compiled here with gcc
    src = r'''
#include <stdio.h>
#include "wdmg.h"
int main(void){printf("%zu %zu %zu %zu\n", sizeof(wdmg_level_params), sizeof(wdmg_mg_params),
 sizeof(wdmg_solve_params), sizeof(wdmg_solve_stats)); return 0;}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.dirname(wdmg.HEADER), c, "-o", exe], check=True)
        sizes = [int(v) for v in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    assert sizes == [ctypes.sizeof(wdmg.LevelParams), ctypes.sizeof(wdmg.MgParams),
                     ctypes.sizeof(wdmg.SolveParams), ctypes.sizeof(wdmg.SolveStats)]


def test_kernel_ids_match_the_header():
    import re
    with open(wdmg.HEADER) as fh:
        text = fh.read()
    body = re.search(r"enum \{\s*(WDMG_K_DSLASH_F64[^}]*)\}", text).group(1)
    names = [n.strip() for n in body.replace("\n", " ").split(",") if n.strip()]
    names = [n.split("=")[0].strip() for n in names]
    assert names[-1] == "WDMG_K_COUNT"
    assert [n[len("WDMG_K_"):].lower() for n in names[:-1]] == wdmg.KERNELS


def test_tuning_keys_match_the_header():
    import re
    with open(wdmg.HEADER) as fh:
        text = fh.read()
    body = re.search(r"enum \{\s*(WDMG_TUNE_AUTO[^}]*)\}", text).group(1)
    vals = {}
    for item in body.replace("\n", " ").split(","):
        item = item.strip()
        if "=" in item:
            k, v = (t.strip() for t in item.split("="))
            vals[k] = int(v)
    assert vals["WDMG_TUNE_AUTO"] == -1
    keys = {k[len("WDMG_TUNE_"):].lower(): v for k, v in vals.items() if k not in ("WDMG_TUNE_AUTO",)}
    assert keys == wdmg.Context.TUNE
    assert "WDMG_TUNE_COUNT" in body and max(keys.values()) + 1 == len(keys)


def test_allocator_callbacks_never_raise_into_the_library():
    """A raising torch allocator must reach the library as NULL (reported as
    WDMG_ERR_OOM), never as an undefined pointer; a raising release is
    swallowed.  Called through the C function pointers ctypes builds."""

    def boom(*_a):
        raise RuntimeError("out of memory")

    alloc, free = wdmg._torch_allocator(boom, boom, 0, None)
    a_cb, f_cb = wdmg._ALLOC_FN(alloc), wdmg._FREE_FN(free)
    a_c = wdmg._ALLOC_FN(ctypes.cast(a_cb, ctypes.c_void_p).value)
    f_c = wdmg._FREE_FN(ctypes.cast(f_cb, ctypes.c_void_p).value)
    for _ in range(100):
        assert a_c(1 << 40, None) is None
    f_c(4096, None)
    ok, _ = wdmg._torch_allocator(lambda n, d, s: 4096 * n, boom, 0, None)
    ok_c = wdmg._ALLOC_FN(ok)
    assert wdmg._ALLOC_FN(ctypes.cast(ok_c, ctypes.c_void_p).value)(3, None) == 3 * 4096


def test_2d_struct_layouts_match_the_binding():
    # wdmg_2d.h compiled as C with gcc: the parameter and statistics structs
    # have the sizes and field offsets the ctypes binding assumes
    from paper_0811_4331_amd import qed2d
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "wdmg_2d.h"
int main(void){printf("%zu %zu %zu %zu %zu\n", sizeof(wdmg_2d_mg_params), sizeof(wdmg_2d_stats),
 offsetof(wdmg_2d_mg_params, omega), offsetof(wdmg_2d_mg_params, blocking), offsetof(wdmg_2d_stats, flops));
 return 0;}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.dirname(wdmg.HEADER), c, "-o", exe], check=True)
        got = [int(v) for v in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    assert got == [ctypes.sizeof(qed2d.MgParams2d), ctypes.sizeof(qed2d.Stats2d), qed2d.MgParams2d.omega.offset,
                   qed2d.MgParams2d.blocking.offset, qed2d.Stats2d.flops.offset]


def test_2d_create_rejects_bad_dims_without_a_gpu_call():
    from paper_0811_4331_amd import qed2d
    lib = qed2d.load()
    h = ctypes.c_void_p()
    for dims in ((3, 8), (8, 2), (6, 7)):
        assert lib.wdmg_2d_create(ctypes.byref(h), (ctypes.c_int * 2)(*dims), None, None) == -2
    assert lib.wdmg_2d_create(None, (ctypes.c_int * 2)(8, 8), None, None) == -1


def test_2d_entry_points_reject_a_null_context_without_a_gpu_call():
    from paper_0811_4331_amd import qed2d
    lib = qed2d.load()
    null = None
    assert lib.wdmg_2d_set_gauge(null, null, -1) == -1
    assert lib.wdmg_2d_set_mass(null, 0.1) == -1
    assert lib.wdmg_2d_apply_D(null, null, null, 1, 0) == -1
    assert lib.wdmg_2d_mg_setup(null, None) == -1
    assert lib.wdmg_2d_get_prolongator(null, 0, null) == -1
    assert lib.wdmg_2d_apply_coarse(null, 1, null, null, 1) == -1
    assert lib.wdmg_2d_restrict(null, 0, null, null, 1) == -1
    assert lib.wdmg_2d_prolong(null, 0, null, null, 1) == -1
    assert lib.wdmg_2d_get_coarse_operator(null, 1, null) == -1
    assert lib.wdmg_2d_vcycle(null, null, null) == -1
    assert lib.wdmg_2d_solve(null, null, null, 0, 1e-10, 10, None) == -1
    assert lib.wdmg_2d_last_error(null) == b"null context"
    lib.wdmg_2d_destroy(null)
