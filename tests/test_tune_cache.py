"""The tuner's cache file handling (host only, no GPU): entries for a key are
replaced, other entries kept, and the library's reader format (eleven fields, '#'
comments) is what the tuner writes."""
import paper_2512_12232_amd.tune as T


def test_write_entries_replaces_only_its_keys(tmp_path):
    p = tmp_path / "c.txt"
    T.write_entries(str(p), [["gfx950", 1024, 512, 0, 0, 5, 1, 2, 0, 0, 0, "a"],
                             ["gfx950", 0, 0, 2, 1, 0, 1, 0, 0, 4, 64]], "first")
    T.write_entries(str(p), [["gfx950", 1024, 512, 0, 0, 4, 2, 0, 0, 0, 0, "b"]], "second")
    rows = [l.split("#")[0].split() for l in p.read_text().splitlines()
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 2 and all(len(r) == 11 for r in rows)
    keyed = {tuple(r[:5]): r[5:] for r in rows}
    assert keyed[("gfx950", "1024", "512", "0", "0")] == ["4", "2", "0", "0", "0", "0"]
    assert keyed[("gfx950", "0", "0", "2", "1")] == ["0", "1", "0", "0", "4", "64"]


def test_shipped_cache_parses():
    rows = [l.split("#")[0].split() for l in open(T.DEFAULT_CACHE).read().splitlines()
            if l.strip() and not l.startswith("#")]
    assert rows and all(len(r) == 11 for r in rows)
    for r in rows:
        nx, ny, prec, batched, hc, em, sm, lb, tpw, ipl = (int(v) for v in r[1:])
        assert hc in (0, 4, 5, 8) and em in (0, 1, 2) and sm in (0, 1, 2)
        assert lb % 8 == 0 and 0 <= lb <= 1024 and 0 <= tpw <= 64 and batched in (0, 1)
