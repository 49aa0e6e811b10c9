"""Walk programs compile for gfx950 through the C ABI (runtime compilation
against csrc/program_rt.hpp); no GPU needed.  A broken program reports the
compiler's message."""
import pytest

from paper_2107_11983_amd import TrwError, check_program, programs

SOURCES = {
    **{f"deepwalk-{s}": programs.deepwalk(s) for s in ("naive", "alias", "its", "rej")},
    **{f"ppr-{s}": programs.ppr(s) for s in ("naive", "alias", "its", "rej")},
    "node2vec": programs.NODE2VEC,
    "metapath": programs.METAPATH,
    "weighted-node2vec": programs.WEIGHTED_NODE2VEC,
    "node2vec-its": programs.NODE2VEC_ITS,
    "weighted-rej": programs.WEIGHTED_REJ,
}


@pytest.mark.parametrize("name", sorted(SOURCES))
def test_program_compiles(name):
    check_program(SOURCES[name], "gfx950")


def test_broken_program_reports_the_compiler():
    bad = programs.NODE2VEC.replace("return false;", "return undefined_name;")
    with pytest.raises(TrwError) as ei:
        check_program(bad, "gfx950")
    assert "undefined_name" in str(ei.value)
