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


def test_committed_profiles_match_the_kernel_sources():
    """The rocprofv3 summaries under profiles/ that record a kernel-source hash
    were taken from the current kernel sources (else bench.py reports no HBM
    traffic and the summaries describe other code)."""
    import glob
    import os
    paths = sorted(glob.glob(os.path.join(bench.ROOT, "profiles", "*.txt")))
    stamped = 0
    for p in paths:
        for line in open(p):
            if line.startswith("kernel_source_sha256:"):
                stamped += 1
                assert line.split(":", 1)[1].strip() == bench.kernel_source_hash(), os.path.basename(p)
    assert stamped >= 1
