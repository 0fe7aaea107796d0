"""The rocprofv3 summary tool used for the committed profiles (no GPU)."""
import csv

from paper_2310_00810_amd import profiling as P


def _trace(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, s, e in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": s, "End_Timestamp": e})


def test_overlap_split(tmp_path):
    # a: alone 0-10 us; b overlaps c (20-40 us and 30-35 us); a again alone 50-56 us; c nested in b
    _trace(tmp_path / "t.csv", [
        ("void lbm::k_a<19, 0>(lbm::Geo)", 0, 10_000),
        ("void lbm::k_b(lbm::Geo)", 20_000, 40_000),
        ("void lbm::k_c(lbm::Geo)", 30_000, 35_000),
        ("void lbm::k_a<19, 0>(lbm::Geo)", 50_000, 56_000),
    ])
    out = tmp_path / "o.md"
    out.write_text("")
    P.overlap(str(tmp_path / "t.csv"), str(out))
    rows = {}
    for line in out.read_text().splitlines():
        if line.startswith("| `"):
            cells = [c.strip() for c in line.strip("|").split("|")]
            rows[cells[0].strip("`")] = cells[1:]
    assert rows["k_a<19, 0>"] == ["2", "8.00", "0", "0.00"]
    assert rows["k_b"] == ["0", "0.00", "1", "20.00"]
    assert rows["k_c"] == ["0", "0.00", "1", "5.00"]


def test_overlap_chain(tmp_path):
    # E overlaps F, F overlaps L, L overlaps C; E does not overlap C, and G stands alone
    _trace(tmp_path / "t.csv", [("k_e", 0, 50), ("k_f", 5, 60), ("k_l", 55, 200), ("k_c", 56, 57),
                                ("k_g", 300, 310)])
    out = tmp_path / "o.md"
    out.write_text("")
    P.overlap(str(tmp_path / "t.csv"), str(out))
    text = out.read_text()
    for k in ("k_e", "k_f", "k_l", "k_c"):
        assert f"| `{k}` | 0 |" in text, k
    assert "| `k_g` | 1 |" in text


def test_short_names():
    assert P.short_name("void lbm::k_step<19, 0>(lbm::Geo, float const*)") == "k_step<19, 0>"
    assert P.short_name("void nn::k_wgrad<true>(nn::ConvArgs)") == "k_wgrad<true>"


def test_mfma_summary_rates(tmp_path):
    """One dispatch of 10 us with 1 000 wavefronts of 10 000 BF16 MOPS each:
    5.12 GFLOP in 10 us = 512 TFLOP/s, 0.205 of the dense peak; MFMA busy
    from cycles summed over the 8 XCDs."""
    path = tmp_path / "c.csv"
    fields = ["Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    gui = 8 * 2.4e9 * 10e-6                     # 8 XCDs x 2.4 GHz x 10 us
    vals = {"SQ_WAVES": 1000, "SQ_INSTS_VALU_MFMA_MOPS_BF16": 1000 * 10_000, "GRBM_GUI_ACTIVE": gui,
            "SQ_VALU_MFMA_BUSY_CYCLES": 0.25 * gui / 8 * 1024, "SQ_INSTS_LDS": 2000, "SQ_LDS_BANK_CONFLICT": 1000,
            "SQ_WAIT_INST_LDS": 5000}
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for name, v in vals.items():
            w.writerow({"Kernel_Name": "void nn::k_wgrad_halo<32, 1, 4>(nn::ConvArgs)", "Counter_Name": name,
                        "Counter_Value": v, "Start_Timestamp": 0, "End_Timestamp": 10_000})
    out = tmp_path / "m.md"
    P.mfma(str(path), str(out), "cmd")
    row = [ln for ln in out.read_text().splitlines() if ln.startswith("| `k_wgrad_halo")][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1:] == ["1", "1000", "10.0", "512", "0.205", "0.250", "2.0", "0.50", "5"]
