"""The kernel-trace summaries behind profiles/: grouping by kernel and launch
shape, and the listing of one apply (the kernels after the next-to-last
tau-stream launch), on a small rocpd-like database written here."""
import sqlite3
import subprocess
import sys


def _db(path):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, grid_x int, workgroup_x int, lds_size int, "
                "vgpr_count int, accum_vgpr_count int, duration int, start int)")
    rows = []
    t = 0
    for apply in range(3):
        for name, gx, du in (("void bsex::k_gather<double2>(int)", 256, 700_000),
                             ("void bsex::k_dgemm<0, 1, 64>(long)", 512, 1_400_000),
                             ("void bsex::k_tau_stream<2, 4, true, double>(double*)", 1024,
                              78_000_000)):
            rows.append((name, gx, 256, 0, 64, 0, du + apply, t))
            t += du + 10
    con.executemany("insert into kernels values (?,?,?,?,?,?,?,?)", rows)
    con.commit()
    con.close()


def _run(*args):
    return subprocess.run([sys.executable, "-m", "paper_2607_20728_amd.profsummary", *args],
                          capture_output=True, text=True, check=True).stdout


def test_kernels_and_last_apply(tmp_path):
    db = str(tmp_path / "t_results.db")
    _db(db)
    out = _run("kernels", db, "10").splitlines()
    assert out[0].split()[0] == "kernel"
    first = out[1].split()
    assert first[0] == "k_tau_stream<2," and first[-4] == "3"        # 3 calls, largest total
    assert abs(float(first[-3]) - 78000.0) < 0.1                      # mean duration in us
    apply = _run("apply", db).splitlines()
    names = [line.split()[0] for line in apply[1:]]
    assert names == ["k_gather<double2>", "k_dgemm<0,", "k_tau_stream<2,"]
