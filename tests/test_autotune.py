"""CPU tests of the autotuner's table handling (no GPU: lookup and table form)."""
from paper_2303_02317_amd import autotune


def table():
    recs = {}
    for (m, lg, p, pub) in ((0, 14, 0, 11), (0, 20, 0, 12), (1, 16, 0, 13), (1, 16, 1, 11)):
        recs[autotune.class_key(m, lg, p)] = dict(model=m, lg=lg, precision=p,
                                                  best=dict(pub_min_lg=pub, direct_max_h=160, direct_max_n=1024))
    return {"arch": "gfx950", "classes": recs}


def test_lookup_nearest_class_of_the_same_model():
    t = table()
    assert autotune.lookup(t, 0, 2 ** 14)["pub_min_lg"] == 11
    assert autotune.lookup(t, 0, 2 ** 19)["pub_min_lg"] == 12      # nearest log2 T is 20
    assert autotune.lookup(t, 0, 3000)["pub_min_lg"] == 11         # ceil(log2 3000) = 12 -> 14
    assert autotune.lookup(t, 1, 2 ** 16, precision=1)["pub_min_lg"] == 11
    assert autotune.lookup(t, 1, 2 ** 16, precision=0)["pub_min_lg"] == 13
    assert autotune.lookup(t, 2, 2 ** 16) is None                   # no BSM class tuned


def test_server_table_lists_every_class():
    rows = autotune.server_table(table())
    assert sorted((m, lg, p) for m, lg, p, _ in rows) == [(0, 14, 0), (0, 20, 0), (1, 16, 0), (1, 16, 1)]


def test_candidates_cover_the_tuned_fields():
    keys = set(autotune.SCHEDULE_KEYS)
    assert all(set(dict(autotune.SCHEDULE_DEFAULTS, **c)) == keys for c in autotune.CANDIDATES)
    assert keys <= {"workgroups", "pub_min_lg", "pub_direct", "direct_max_h", "direct_max_n", "helper_idle_us",
                    "timeout_ms", "timeout_us", "lds_max_lg", "radix_lg"}
    # FFT schedules are among the candidates: LDS transform size and pass radix
    assert {dict(autotune.SCHEDULE_DEFAULTS, **c)["lds_max_lg"] for c in autotune.CANDIDATES} == {11, 12}
    assert {dict(autotune.SCHEDULE_DEFAULTS, **c)["radix_lg"] for c in autotune.CANDIDATES} == {2, 3}


def test_committed_table_is_well_formed():
    t = autotune.load_cache()
    for key, rec in t.get("classes", {}).items():
        assert key == autotune.class_key(rec["model"], rec["lg"], rec["precision"])
        assert set(rec["best"]) <= set(autotune.SCHEDULE_KEYS)
