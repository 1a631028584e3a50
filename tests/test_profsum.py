"""Host logic of the profile summariser: counter means per kernel and the
copy-calibrated traffic figure, on small synthetic rocprofv3-style CSV files."""
import csv

from paper_2105_11788_amd import profsum

COLS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(COLS)
        w.writerows(rows)


def test_counter_means_by_kernel(tmp_path):
    p = tmp_path / "c.csv"
    write(p, [[1, "k_a(int)", "FETCH_SIZE", 10.0], [2, "k_a(int)", "FETCH_SIZE", 30.0],
              [3, "k_b(int)", "FETCH_SIZE", 5.0]])
    m = profsum.counter_means(str(p))
    assert m[("k_a(int)", "FETCH_SIZE")] == (2, 20.0)
    assert m[("k_b(int)", "FETCH_SIZE")] == (1, 5.0)
    assert set(profsum.counter_means(str(p), "k_b")) == {("k_b(int)", "FETCH_SIZE")}


def test_traffic_calibration(tmp_path, capsys):
    # a copy of 1 MiB whose FETCH_SIZE reads half and WRITE_SIZE all of it
    write(tmp_path / "fc.csv", [[1, "k_copy16(x)", "FETCH_SIZE", 512.0]])
    write(tmp_path / "wc.csv", [[1, "k_copy16(x)", "WRITE_SIZE", 1024.0]])
    write(tmp_path / "f.csv", [[1, "k_x(y)", "FETCH_SIZE", 100.0], [2, "k_x(y)", "FETCH_SIZE", 300.0]])
    write(tmp_path / "w.csv", [[1, "k_x(y)", "WRITE_SIZE", 50.0]])
    (tmp_path / "src").mkdir()
    (tmp_path / "src" / "a.hip").write_text("kernel")
    profsum.main(["traffic", "--kernel", "k_x", "--fetch", str(tmp_path / "f.csv"),
                  "--write", str(tmp_path / "w.csv"), "--copy-fetch", str(tmp_path / "fc.csv"),
                  "--copy-write", str(tmp_path / "wc.csv"), "--copy-bytes", str(1 << 20),
                  "--sources", str(tmp_path / "src")])
    kv = dict(line.split(": ", 1) for line in capsys.readouterr().out.strip().splitlines())
    assert float(kv["fetch_factor"]) == 2.0 and float(kv["write_factor"]) == 1.0
    # (2 x 200 KiB + 1 x 50 KiB) per launch
    assert int(kv["traffic_bytes_per_launch"]) == (2 * 200 + 50) * 1024
    assert kv["source_sha1"] == profsum.source_digest(str(tmp_path / "src"))


def test_source_digest_tracks_changes(tmp_path):
    (tmp_path / "k.hip").write_text("a")
    d1 = profsum.source_digest(str(tmp_path))
    (tmp_path / "k.hip").write_text("b")
    assert profsum.source_digest(str(tmp_path)) != d1


def test_source_digest_of_listed_files_ignores_the_others(tmp_path):
    (tmp_path / "k.hip").write_text("a")
    (tmp_path / "other.hip").write_text("x")
    d1 = profsum.source_digest(str(tmp_path), ["k.hip"])
    (tmp_path / "other.hip").write_text("y")
    assert profsum.source_digest(str(tmp_path), ["k.hip"]) == d1
    (tmp_path / "k.hip").write_text("b")
    assert profsum.source_digest(str(tmp_path), ["k.hip"]) != d1
