"""bench.py's contract that needs no GPU: more than one GPU is refused with
a message before any device work, and the committed counter summary that
feeds the roofline's traffic field parses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_committed_traffic_summary_parses():
    sys.path.insert(0, ROOT)
    import bench
    tr = bench.read_traffic(os.path.join(ROOT, "profiles", "traffic_wedge512.txt"))
    assert tr is not None
    assert len(tr["kernel_source_sha"]) == 16
    # pass B with density classes on 128x4 plane tiles, the kernel the
    # roofline reports at 512^3
    assert float(tr["bytes[k_iter<0, 2, 3>]"]) > 0
    # the kernel-trace summary gives the command it came from
    stats = open(os.path.join(ROOT, "profiles", "kernel_stats_wedge512.txt")).read()
    assert "rocprofv3 --kernel-trace --stats" in stats and "k_iter<0, 2, 3>" in stats


def test_launch_filters():
    """The summaries' launch filters: the median is taken over the non-empty
    launches even when empty ones (the end of a captured chunk) are the
    majority, and the two forms of the iteration are told apart although a
    few much longer set-up launches stretch the range."""
    sys.path.insert(0, ROOT)
    from paper_1410_1942_amd import profiling as pr
    vals = [0.0] * 70 + [1.0, 1.0, 2.0] * 20
    big = pr._large(vals)
    assert len(big) == 60 and min(big) == 1.0
    forms = [1.0] * 200 + [1.46] * 100 + [2.65] * 3
    (na, ma), (nb, mb) = pr._two_forms(forms)
    assert na == 200 and ma == 1.0
    assert nb == 103 and 1.46 < mb < 1.5


def test_trace_segments(tmp_path):
    """A trace cut at idle gaps: the runs of matching launches are told apart
    and one of them is summarized alone."""
    sys.path.insert(0, ROOT)
    from paper_1410_1942_amd import profiling as pr
    rows = ["Kernel_Name,Start_Timestamp,End_Timestamp"]
    t = 0
    for run, n in ((0, 3), (1, 5)):
        for i in range(n):
            rows.append(f'"k_iter<1, 2, 1>(run{run})",{t},{t + 1000 * (run + 1)}')
            rows.append(f'"k_other",{t + 10},{t + 20}')
            t += 100_000
        t += 10_000_000                      # 10 ms without a matching launch
    path = tmp_path / "trace.csv"
    path.write_text("\n".join(rows) + "\n")
    first = pr.kernel_stats(str(path), "k_iter<1,", 2.0, 0)
    assert "3 launches" in first and "run1" not in first and "k_other" not in first
    second = pr.kernel_stats(str(path), "k_iter<1,", 2.0, 1)
    assert "5 launches" in second and "run0" not in second
    assert "k_other" in pr.kernel_stats(str(path))
