"""The profile summariser's kernel names and stats table (CPU)."""
import csv

from paper_1807_00399_amd import rocprof_summary as rs


def test_kernel_names_keep_literal_template_arguments():
    assert rs._short("_ZN3pcg12_GLOBAL__N_113k_enc_forwardILb0EEEvPKfS3_PKlPKiiiPKdS3_S3_PKDF16bSB_PfPi") == \
        "pcg::k_enc_forward<false>"
    assert rs._short("_ZN3pcg12_GLOBAL__N_113k_enc_forwardILb1EEEvPKf") == "pcg::k_enc_forward<true>"
    assert rs._short("_ZN3pcg12_GLOBAL__N_15k_knnILi16ELi8EEEvNS_8GridViewEPKfliPiPf") == "pcg::k_knn<16, 8>"
    assert rs._short("void pcg::(anonymous namespace)::k_icp_accum<64, 8, 0>(pcg::GridView)") == \
        "pcg::k_icp_accum<64, 8, 0>"


def test_stats_table(tmp_path):
    src = tmp_path / "ks.csv"
    with open(src, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs",
                                          "Percentage"])
        w.writeheader()
        w.writerow({"Name": "_ZN3pcg12_GLOBAL__N_113k_enc_forwardILb0EEEvPKf", "Calls": 4,
                    "TotalDurationNs": 1200000, "AverageNs": 300000, "MinNs": 290000, "MaxNs": 310000,
                    "Percentage": 75.0})
    out = tmp_path / "out.txt"
    rs.stats(str(src), str(out), "the command")
    lines = out.read_text().splitlines()
    assert lines[1] == "# command: the command"
    assert lines[3].split() == ["4", "1200.0", "300.00", "290.00", "310.00", "75.00", "pcg::k_enc_forward<false>"]
