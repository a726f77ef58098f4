"""The rocprofv3 summary tool: counter scaling by the copy calibration, the
machine-readable traffic lines that bench.py reads, and the source digest
that voids them when the kernels change."""
import csv

from paper_2602_08982_amd import profsum as P


def _write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_counters_summary_and_traffic_lookup(tmp_path, monkeypatch):
    lap2 = "void tdslda::k_lap2<double, 32, 32, 32, 3, 4, 5>(tdslda::Lap2Args<double>)"
    copy = "__amd_rocclr_copyBuffer"
    # the copy reads 2^32 bytes and FETCH_SIZE reports half of them (KiB)
    fetch = [(copy, "FETCH_SIZE", 2 ** 31 / 1024), (lap2, "FETCH_SIZE", 1000.0), (lap2, "FETCH_SIZE", 3000.0)]
    write = [(copy, "WRITE_SIZE", 2 ** 32 / 1024), (lap2, "WRITE_SIZE", 500.0), (lap2, "WRITE_SIZE", 500.0)]
    fp, wp, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "c.md"
    _write_counters(fp, fetch)
    _write_counters(wp, write)

    class A:
        pass

    a = A()
    a.fetch, a.write, a.out, a.command, a.title, a.note = str(fp), str(wp), str(out), ["cmd"], "t", ""
    P.cmd_counters(a)
    # read: 2 x mean(1000, 3000) KiB; written: 1 x 500 KiB
    want = (2 * 2000.0 + 500.0) * 1024
    got = P.read_traffic(str(out), "double", 32, "lap2_full")
    assert abs(got - want) < 1e-6 * want
    assert P.read_traffic(str(out), "double", 48, "lap2_full") is None
    monkeypatch.setattr(P, "sources_digest", lambda: "0" * 16)
    assert P.read_traffic(str(out), "double", 32, "lap2_full") is None


def test_roles_and_keys():
    assert P.role("void tdslda::k_lap2<float, 48, 48, 48, 2, 4, 5>(tdslda::Lap2Args<float>)") == "lap2_corr"
    assert P.key("void tdslda::k_lap1<double, 32, 1024, 64>(...)") == "double:32:lap1"
    assert P.key("void tdslda::(anonymous namespace)::q_lap2<float, 16, 64, 3, 4, 5>(...)") == "float:16:q1d_lap2_full"
    assert P.key("tdslda::k_finalize(long, tdslda::StateScalars, int)") == ":-:finalize"
    assert P.role("rocsolver::v33001::stedc_solve_kernel<double>(int)") is None
    assert P.key("void tdslda::(anonymous namespace)::q_gen<float, 16, 256, 3, 4, 5>(...)") == "float:16:q1dgen_lap2_full"
    assert P.role("void tdslda::(anonymous namespace)::q_gen<float, 16, 256, 5, 4, 5>(...)") == "q1dgen_lap1"
    assert P.role("void tdslda::(anonymous namespace)::q_densj<float, 16, 512, 256>(...)") == "q1dgen_dens"


def test_library_copy_calibrates(tmp_path):
    """The library's own 4 GiB streaming copy is the calibration dispatch
    (the largest k_stream_copy reading)."""
    agg = {"tdslda::k_stream_copy(cp_v4i const*, cp_v4i*, long)": [2 ** 31 / 1024 * 1024.0, 100.0]}
    assert abs(P._copy_factor(agg) - 2.0) < 1e-12


def test_sq_summary_normalisation(tmp_path):
    """One dispatch of 1 ms at a 2 GHz GRBM clock (8 XCDs): the wave-cycle,
    VALU and LDS counters (quad-cycles) become waves per CU and busy
    fractions, the conflict counter a rate per LDS-active cycle."""
    lap2 = "void tdslda::k_lap2<double, 32, 32, 32, 2, 4, 5>(tdslda::Lap2Args<double>)"
    cyc = 2e9 * 1e-3
    vals = {"GRBM_GUI_ACTIVE": 8 * cyc, "SQ_WAVE_CYCLES": 256 * cyc * 12 / 4, "SQ_ACTIVE_INST_VALU": 1024 * cyc * 0.5 / 4,
            "SQ_ACTIVE_INST_LDS": 256 * cyc * 0.25 / 4, "SQ_LDS_BANK_CONFLICT": 256 * cyc * 0.25 / 4 * 0.3,
            "SQ_WAVES": 1000.0, "SQ_INSTS_VALU": 1.5e6}
    p, out = tmp_path / "sq.csv", tmp_path / "sq.md"
    with open(p, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"])
        for k, v in vals.items():
            w.writerow([1, lap2, k, v, 0, 1000000])

    class A:
        pass

    a = A()
    a.csv, a.out, a.command, a.title, a.note = str(p), str(out), ["cmd"], "t", ""
    P.cmd_sq(a)
    row = [ln for ln in open(out) if "lap2_corr" in ln][0].split("|")
    assert [c.strip() for c in row[3:11]] == ["1", "1.000", "2.00", "12.0", "0.50", "1500", "0.250", "0.300"]
