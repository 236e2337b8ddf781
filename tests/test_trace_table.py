"""The launch-size table (trace_table): a kernel trace, a round log and the
two counter files joined by hand-made inputs whose figures are known."""
import csv
import json

from paper_2503_21937_amd import trace_table

K = "void dlfix::k_window_round<unsigned int, 1, 4, 2>(dlfix::JoinArgs, dlfix::DenseArgs, dlfix::RoundArgs)"


def write_trace(path, durs_us):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        t = 1000
        w.writerow(["dlfix::k_fill32(unsigned int*, unsigned long, unsigned int)", t, t + 5000])
        for d in durs_us:
            t += 100000
            w.writerow([K, t, t + int(d * 1000)])


def write_counter(path, name, kib):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, v in enumerate(kib):
            w.writerow([10 + i, K, name, v])
            w.writerow([10 + i, "other", name, 999.0])


def test_classes_rates_and_traffic(tmp_path):
    trace, log = tmp_path / "t.csv", tmp_path / "log.jsonl"
    # an earlier launch (not in the log), then rounds of 0, 50, 2e6 and 3e7 derivations
    write_trace(trace, [7.0, 10.0, 20.0, 40.0, 100.0])
    log.write_text(json.dumps({"semiring": "maxmin", "driver_rows": 1000, "bytes_per_unit": 8,
                               "derivations": [30_000_000, 2_000_000, 50, 0]}) + "\n")
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counter(fetch, "FETCH_SIZE", [1.0, 1000.0, 2000.0, 30.0, 4.0])
    write_counter(write, "WRITE_SIZE", [1.0, 500.0, 1000.0, 10.0, 2.0])
    out = trace_table.main(str(trace), str(log), str(fetch), str(write), 2.0, 1.0).splitlines()
    rows = {r.split("|")[1].strip(): [c.strip() for c in r.split("|")[2:-1]] for r in out[2:]}
    # log order = launch order of the last four launches: 3e7 -> 10 us, 2e6 -> 20, 50 -> 40, 0 -> 100
    big = rows[">= 1e7"]
    assert big[0] == "1" and big[1] == "10.0"
    b = (1000 + 30_000_000) * 8
    assert big[4] == f"{b / 1e6:.2f}" and big[5] == f"{b / 10e-6 / 1e9:.0f}"
    assert big[7] == f"{(1000.0 * 2 + 500.0) * 1024 / 1e6:.2f}"
    assert rows["1e6 .. 1e7"][1] == "20.0" and rows["1 .. 1e5"][1] == "40.0"
    assert rows["0 (after the last round)"][1] == "100.0"
    assert "1e5 .. 1e6" not in rows
    assert rows["all"][0] == "4" and rows["all"][3] == "100.0%"


def test_log_longer_than_trace_is_refused(tmp_path):
    trace, log = tmp_path / "t.csv", tmp_path / "log.jsonl"
    write_trace(trace, [1.0])
    log.write_text(json.dumps({"driver_rows": 1, "bytes_per_unit": 8, "derivations": [1, 2]}) + "\n")
    try:
        trace_table.main(str(trace), str(log))
    except SystemExit as e:
        assert "log has 2 launches" in str(e)
    else:
        raise AssertionError("expected a refusal")
