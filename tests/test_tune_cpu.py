"""Autotuner cache (host logic of the C library; no GPU needed)."""

import pytest

from paper_1705_02403_amd import gmt

E, DI = gmt.GMT_COST_EUCLIDEAN, gmt.GMT_COST_DOUBLE_INTEGRATOR


@pytest.fixture(autouse=True)
def clean_cache():
    gmt.gmt_tune_clear()
    yield
    gmt.gmt_tune_clear()


def test_store_lookup_by_bucket():
    gmt.gmt_tune_store(gmt.tune_shape(DI, 6, 16384, 40, 1024), lanes=8, team_wgs=2, workgroups=512, threads=512)
    # same bucket: n in (8192, 16384], m in [32, 63], batch in (512, 1024]
    hit = gmt.gmt_tune_lookup(gmt.tune_shape(DI, 6, 9000, 33, 600))
    assert (hit["lanes"], hit["team_wgs"], hit["workgroups"], hit["threads"]) == (8, 2, 512, 512)
    for other in [gmt.tune_shape(DI, 6, 16385, 40, 1024),   # next n bucket
                  gmt.tune_shape(DI, 6, 16384, 64, 1024),   # next m bucket
                  gmt.tune_shape(DI, 6, 16384, 40, 0),      # single-plan mode
                  gmt.tune_shape(E, 3, 16384, 40, 1024)]:   # other kind
        miss = gmt.gmt_tune_lookup(other)
        assert miss["lanes"] == 0 and miss["team_wgs"] == 0


def test_save_load_round_trip(tmp_path):
    a = gmt.tune_shape(E, 2, 2000, 20, 0)
    b = gmt.tune_shape(DI, 6, 16384, 40, 256)
    gmt.gmt_tune_store(a, 32, 128, threads=1024)
    gmt.gmt_tune_store(b, 4, 1, 0)
    f = tmp_path / "tune.txt"
    gmt.gmt_tune_save(str(f))
    gmt.gmt_tune_clear()
    assert gmt.gmt_tune_lookup(a)["lanes"] == 0
    gmt.gmt_tune_load(str(f))
    assert (gmt.gmt_tune_lookup(a)["lanes"], gmt.gmt_tune_lookup(a)["team_wgs"]) == (32, 128)
    assert gmt.gmt_tune_lookup(a)["threads"] == 1024
    assert gmt.gmt_tune_lookup(b)["lanes"] == 4


@pytest.mark.parametrize("line", [
    "0 2 11 5 0 0 12 64 0 256 1.0 1.0",      # lanes 12 is not a kernel variant
    "0 2 11 5 0 0 16 64 0 256 1.0",          # missing field
    "7 2 11 5 0 0 16 64 0 256 1.0 1.0",      # unknown cost kind
    "0 2 11 5 0 0 16 -1 0 256 1.0 1.0",      # negative team size
    "0 2 11 5 0 0 16 64 0 300 1.0 1.0",      # no 300-thread workgroups
    "0 2 11 5 0 0 16 64 0 256 1.0 1.0 x",    # trailing text
])
def test_malformed_file_loads_nothing(tmp_path, line):
    good = "0 2 11 5 0 0 16 64 0 256 1.0 1.0"
    f = tmp_path / "bad.txt"
    f.write_text("# header\n" + good.replace(" 2 11", " 3 11") + "\n" + line + "\n")
    with pytest.raises(gmt.GmtError):
        gmt.gmt_tune_load(str(f))
    assert gmt.gmt_tune_lookup(gmt.tune_shape(E, 3, 2000, 20, 0))["lanes"] == 0


def test_invalid_store_rejected():
    with pytest.raises(gmt.GmtError):
        gmt.gmt_tune_store(gmt.tune_shape(E, 2, 2000, 20, 0), lanes=12, team_wgs=1)
    with pytest.raises(gmt.GmtError):
        gmt.gmt_tune_store(gmt.tune_shape(E, 9, 2000, 20, 0), lanes=8, team_wgs=1)


def test_build_tiles_in_the_tune_file(tmp_path):
    """Euclidean build-tile lines ("build dim nlog tile ms default_ms") load
    and save with the plan knobs; malformed ones are refused whole."""
    f = tmp_path / "t.txt"
    f.write_text("# header\nbuild 3 14 2 1.250000 1.300000\nbuild 2 11 1 0.100000 0.100000\n")
    gmt.gmt_tune_load(str(f))
    g = tmp_path / "u.txt"
    gmt.gmt_tune_save(str(g))
    text = g.read_text()
    assert "build 3 14 2 1.250000 1.300000" in text and "build 2 11 1 " in text
    gmt.gmt_tune_clear()
    gmt.gmt_tune_save(str(g))
    assert "build" not in g.read_text().split("\n", 1)[1]
    for bad in ("build 3 14 5 1.0 1.0", "build 4 14 1 1.0 1.0", "build 3 14 1 1.0", "build 3 14 1 1.0 1.0 x"):
        f.write_text(bad + "\n")
        with pytest.raises(gmt.GmtError):
            gmt.gmt_tune_load(str(f))
