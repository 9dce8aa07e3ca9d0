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


def test_stage_rooflines(tmp_path):
    """The stage table: means over the applies between stream launches, the
    largest-grid launch of each FFT kernel (the K1e Poisson transforms reuse
    the same kernels on a few grids), and the bytes model (72^3 grid, 35
    planes with sphere modes, N_v = 432, N_b = 8, FP64: inverse plane pass
    5.60 GB = X + 1728 grids x 35 planes x 72^2 x 16 B)."""
    db = str(tmp_path / "s_results.db")
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, grid_x int, workgroup_x int, lds_size int, "
                "vgpr_count int, accum_vgpr_count int, duration int, start int)")
    seq = [("k_sphere_inv_ct<72, 72, 1>(x)", 3000, 2_000_000),
           ("k_fft_axis_ct<72, 1>(x)", 9000, 4_000_000),
           ("k_fft_axis_ct<72, 1>(x)", 20, 14_000),
           ("k_dgemm<0, 1, 64>(x)", 100, 1_000_000),
           ("k_tau_stream_qs<2, true, double>(x)", 5000, 50_000_000)]
    rows, t = [], 0
    for _ in range(3):
        for n, gx, du in seq:
            rows.append((n, gx, 256, 0, 0, 0, du, t))
            t += du + 1
    con.executemany("insert into kernels values (?,?,?,?,?,?,?,?)", rows)
    con.commit()
    con.close()
    out = _run("stages", db, "--grid", "72", "72", "72", "--planes", "35", "--npw", "21079",
               "--nv", "432", "--nb", "8", "--prec", "f64", "--stream-bytes", "300e9")
    lines = {ln.split("(`")[0].strip("| ").strip(): ln for ln in out.splitlines() if "(`" in ln}
    inv = lines["inverse plane pass, sphere -> planes"].split("|")
    assert inv[2].strip() == "5.60 GB" and inv[3].strip() == "2.00"
    axis = lines["inverse axis-1 pass"].split("|")
    assert axis[3].strip() == "4.00"                              # the 20-workgroup launch ignored
    stream = lines["tau stream + combine"].split("|")
    assert stream[4].strip() == "6.00 TB/s" and stream[5].strip() == "0.75"
    assert out.startswith("2 applies")


def test_busy_window(tmp_path):
    """Busy time is the union of kernel intervals in the window after the
    last launch of the named kernel; gaps are binned by size."""
    db = str(tmp_path / "b_results.db")
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start int, end int)")
    rows = [("void k_tau_store<double>(int)", 0, 1_000),            # before the window
            ("void k_tau_store<double>(int)", 2_000, 5_000),        # window opens at 5000
            ("void k_a(int)", 5_000, 8_000),
            ("void k_b(int)", 7_000, 9_000),                        # overlaps k_a
            ("void k_a(int)", 9_005, 10_000),                       # 5 ns gap
            ("void k_b(int)", 210_000, 220_000)]                    # 200 us gap
    con.executemany("insert into kernels values (?,?,?)", rows)
    con.commit()
    con.close()
    out = _run("busy", db, "k_tau_store").splitlines()
    # window 5000..220000 = 215 us; busy 4000 + 995 + 10000 ns
    assert out[0].startswith("window 0.2 ms, kernels busy 0.0 ms (7.0%), 4 launches")
    assert out[1].split()[-3] == "1," and out[3].split()[-3] == "1,"
    table = {line.split()[0]: line.split() for line in out[6:]}
    assert table["k_a"][1] == "2" and table["k_b"][1] == "2"


def test_busy_window_between_launches(tmp_path):
    """NAME@k picks the k-th launch; the window ends where `before` starts."""
    db = str(tmp_path / "w_results.db")
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start int, end int)")
    rows = [("void k_mark(int)", 0, 1_000), ("void k_a(int)", 1_000, 5_000),
            ("void k_mark(int)", 5_000, 6_000), ("void k_b(int)", 6_000, 16_000),
            ("void k_mark(int)", 20_000, 21_000)]
    con.executemany("insert into kernels values (?,?,?)", rows)
    con.commit()
    con.close()
    out = _run("busy", db, "k_mark@2", "5", "k_mark@3").splitlines()
    # window 6000..20000 = 14 us, busy 10 us
    assert out[0].startswith("window 0.0 ms, kernels busy 0.0 ms (71.4%), 1 launches")
    out = _run("busy", db, "k_mark@1", "5", "k_mark@2").splitlines()
    assert "(100.0%)" in out[0]
