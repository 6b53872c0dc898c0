"""bench.py's per-cell flop figures are the oracle's op counts (no GPU)."""
import bench


def test_flops_per_cell_match_oracle_count(orc):
    for recon in (0, 1, 2):
        c = orc.count_ops(recon)
        assert bench.FLOPS_PER_CELL[recon] == 3 * sum(c["face"]) + sum(c["cell"])


def test_gpus_above_one_refused(monkeypatch, capsys):
    import sys
    import pytest
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
