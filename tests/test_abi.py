"""The C-ABI library loads and exports every symbol include/fastea.h declares
(no compute call: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fastea.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fea_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def so():
    from paper_2605_18052_amd import fastea
    if not os.path.exists(fastea.LIB_PATH):
        from paper_2605_18052_amd import build
        build.build()
    return ctypes.CDLL(fastea.LIB_PATH)


def test_every_declared_symbol_is_exported(so):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(so, n), n


def test_binding_covers_header():
    from paper_2605_18052_amd import fastea
    assert sorted(fastea.exported_symbols()) == _declared()


def test_version_and_defaults(so):
    from paper_2605_18052_amd import fastea
    assert fastea.lib().fea_version() == 100
    o = fastea.default_options()
    assert o.rounds == 20 and o.iters_per_round == 50 and o.tau_px_init == 128.0
    assert o.lr_decay == 0.9 and o.reset_moments == 1 and o.tile_matches == 0
    assert o.use_graphs == 1 and o.weight_mode == 0
    assert fastea.lib().fea_default_options(None) == fastea.FEA_EINVAL
    assert fastea.lib().fea_status_string(fastea.FEA_ESTATE) == b"call out of order"


def test_struct_sizes_match_c_layout(tmp_path):
    """The ctypes structures have the sizes and field offsets a C compiler
    gives the header's structures."""
    import subprocess
    from paper_2605_18052_amd import fastea
    structs = {"fea_options": fastea.fea_options, "fea_report": fastea.fea_report,
               "fea_info": fastea.fea_info, "fea_ra_options": fastea.fea_ra_options,
               "fea_ta_options": fastea.fea_ta_options}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fastea.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(ln.split() for ln in subprocess.run([str(exe)], check=True, capture_output=True,
                                                    text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)


def test_null_handles_are_rejected(so):
    from paper_2605_18052_amd import fastea
    L = fastea.lib()
    assert L.fea_batch_solve(0, None, None, None) == fastea.FEA_EINVAL
    assert L.fea_batch_solve(1, None, None, None) == fastea.FEA_EINVAL
    assert L.fea_get_scene_convergence(None, None, None) == fastea.FEA_EINVAL
    assert L.fea_step(None, 1) == fastea.FEA_EINVAL
    assert L.fea_begin_round(None, 1.0) == fastea.FEA_EINVAL
    assert L.fea_get_poses(None, None, None, None) == fastea.FEA_EINVAL
    L.fea_destroy(None)


def test_check_options_without_a_gpu(so):
    from paper_2605_18052_amd import fastea
    ok, why = fastea.check_options(fastea.default_options())
    assert ok == fastea.FEA_OK and why == ""
    bad, why = fastea.check_options(fastea.default_options(tile_matches=3000))
    assert bad == fastea.FEA_EINVAL and "tile_matches" in why
    for field, value in (("persistent_steps", 2), ("wait_limit_us", -1)):
        bad, why = fastea.check_options(fastea.default_options(**{field: value}))
        assert bad == fastea.FEA_EINVAL and field in why, (field, why)
    assert fastea.check_options(fastea.default_options(persistent_steps=1, wait_limit_us=10))[0] == fastea.FEA_OK
    assert fastea.lib().fea_check_options(None, None, 0) == fastea.FEA_EINVAL


@pytest.mark.parametrize("tile", [1024, 2048, 4096])
def test_learned_quadratic_form_with_small_items_is_refused(so, tile):
    """Learned weights with the quadratic form accept only the default
    (8192-match) work items; smaller ones are refused before any GPU work."""
    from paper_2605_18052_amd import fastea
    o = fastea.default_options(weight_mode=1, inner_loop=1, tile_matches=tile)
    rc, why = fastea.check_options(o)
    assert rc == fastea.FEA_EINVAL and "tile_matches 0 or 8192" in why
    for t in (0, 8192):
        assert fastea.check_options(fastea.default_options(weight_mode=1, inner_loop=1,
                                                           tile_matches=t))[0] == fastea.FEA_OK
    # each alone stays accepted with small items
    assert fastea.check_options(fastea.default_options(inner_loop=1, tile_matches=tile))[0] == fastea.FEA_OK
    assert fastea.check_options(fastea.default_options(weight_mode=1, tile_matches=tile))[0] == fastea.FEA_OK
