"""Host-side checks of the autotuner's table file (no GPU needed)."""
import pytest


def test_tune_table_roundtrip(tmp_path):
    import paper_1412_1127_amd as ax
    src = tmp_path / "in.txt"
    # a square-class line and a rectangular one
    src.write_text("0 6 12 1 0.600000\n1 1 9 12 12 2 0.080000\n\n")
    ax.accx_tune_load(str(src))
    out = tmp_path / "out.txt"
    ax.accx_tune_save(str(out))
    got = set(out.read_text().split("\n")) - {""}
    assert {"0 6 12 12 12 1 0.600000", "1 1 9 12 12 2 0.080000"} <= got
    # the saved form loads back
    ax.accx_tune_load(str(out))


def test_tune_table_rejects_garbage(tmp_path):
    import paper_1412_1127_amd as ax
    bad = tmp_path / "bad.txt"
    bad.write_text("0 6 12 9 0.1\n")
    with pytest.raises(ax.AccxError):
        ax.accx_tune_load(str(bad))
    for junk in ("0 6 12 12 1 3.5\n", "0 6 12 1 x\n", "0 6 12 1\n", "0 6 12 12 12 1 0.5 7\n"):
        bad.write_text(junk)
        with pytest.raises(ax.AccxError):
            ax.accx_tune_load(str(bad))
    with pytest.raises(ax.AccxError):
        ax.accx_tune_load(str(tmp_path / "missing.txt"))
