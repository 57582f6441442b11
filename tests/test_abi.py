"""The C-ABI library loads and exports every symbol the header declares
(no compute calls: this runs without a GPU)."""
import ctypes as C
import os
import subprocess

import pytest

from paper_2609_31258_amd import mucite


def test_library_exports_every_declared_symbol():
    L = mucite.load_library()
    names = mucite.declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert L.mc_abi_version() == mucite.ABI_VERSION == 6


def test_binding_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "mucite.h"\n#include <stdio.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(mc_options), '
                   'sizeof(mc_grid), sizeof(mc_field_tables), sizeof(mc_ion), sizeof(mc_source), '
                   'sizeof(mc_operating), sizeof(mc_packs), sizeof(mc_tallies), sizeof(mc_exit_rec), '
                   'sizeof(mc_info), sizeof(mc_timing), sizeof(mc_sample_rec), sizeof(mc_tally_layout), '
                   'sizeof(mc_cic_packs));'
                   'return 0;}\n')
    inc = os.path.join(os.path.dirname(mucite.HERE), "include")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I" + inc, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [C.sizeof(s) for s in (mucite.Options, mucite.Grid, mucite.FieldTables, mucite.Ion, mucite.Source,
                                  mucite.Operating, mucite.Packs, mucite.Tallies, mucite.ExitRec, mucite.Info,
                                  mucite.Timing, mucite.SampleRec, mucite.TallyLayout, mucite.CicPacks)]
    assert got == want


def test_serving_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "sz2.c"
    src.write_text('#include "mucite.h"\n#include <stdio.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(mc_server_options), sizeof(mc_query), '
                   'sizeof(mc_query_result), sizeof(mc_server_stats));return 0;}\n')
    inc = os.path.join(os.path.dirname(mucite.HERE), "include")
    exe = tmp_path / "sz2"
    subprocess.run(["gcc", "-I" + inc, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [C.sizeof(s) for s in (mucite.ServerOptions, mucite.Query, mucite.QueryResult, mucite.ServerStats)]
    assert got == want


def test_null_arguments_are_rejected_without_a_device():
    L = mucite.load_library()
    assert L.mc_create(None, None) == mucite.MC_EINVAL
    assert L.mc_step(None, 1) == mucite.MC_EINVAL
    assert L.mc_read_tallies(None, None) == mucite.MC_EINVAL
    assert L.mc_get_tally_layout(None, None) == mucite.MC_EINVAL
    assert L.mc_deposit_cic(None, None, None, None) == mucite.MC_EINVAL
    assert L.mc_deposit_cic_noalloc(None, None, None, None) == mucite.MC_EINVAL
    L.mc_destroy(None)
    assert L.mc_server_submit(None, None, None) == mucite.MC_EINVAL
    assert L.mc_server_poll(None, 1, None) == mucite.MC_EINVAL
    L.mc_server_destroy(None)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises; nothing falls back."""
    monkeypatch.setattr(mucite, "_LIB", None)
    monkeypatch.setattr(mucite, "LIB_PATH", str(tmp_path / "libmucite.so"))
    with pytest.raises(RuntimeError, match="not built"):
        mucite.load_library()
