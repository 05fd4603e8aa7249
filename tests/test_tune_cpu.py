"""Host-side checks of the autotuner's table file (no GPU needed)."""
import pytest


def test_tune_table_roundtrip(tmp_path):
    import paper_1412_1127_amd as ax
    src = tmp_path / "in.txt"
    src.write_text("0 6 12 1 0.600000\n1 1 12 2 0.080000\n")
    ax.accx_tune_load(str(src))
    out = tmp_path / "out.txt"
    ax.accx_tune_save(str(out))
    got = set(out.read_text().split("\n")) - {""}
    assert {"0 6 12 1 0.600000", "1 1 12 2 0.080000"} <= got


def test_tune_table_rejects_garbage(tmp_path):
    import paper_1412_1127_amd as ax
    bad = tmp_path / "bad.txt"
    bad.write_text("0 6 12 9 0.1\n")
    with pytest.raises(ax.AccxError):
        ax.accx_tune_load(str(bad))
    with pytest.raises(ax.AccxError):
        ax.accx_tune_load(str(tmp_path / "missing.txt"))
