"""Host logic of the benchmark: kernel-name mapping, PMC folding with the
copy-kernel calibration, and the algorithmic byte model."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import scenarios  # noqa: E402


def test_kernel_key_mapping():
    k = bench.kernel_key
    assert k("void dnslab::(anonymous namespace)::k_mom_stage<double, 1, true>(dnslab::MomArgs<double>)") == "mom_stage"
    assert k("void dnslab::(anonymous namespace)::k_sca_stage_b<float, 3>(dnslab::BRec<...> const*)") == "scalar_stage"
    assert k("void dnslab::(anonymous namespace)::k_filter_lds<double, 3>(dnslab::FiltArgs<double>)") == "filter"
    assert k("void dnslab::(anonymous namespace)::k_filter<double, 1>(dnslab::FiltArgs<double>)") == "filter_c"
    assert k("void dnslab::(anonymous namespace)::k_fft_cols<double, 2>(dnslab::FFTArgs<double>)") == "fft_z"
    assert k("void dnslab::(anonymous namespace)::k_fft_cols<float, 1>(dnslab::FFTArgs<float>)") == "fft_y"
    assert k("void dnslab::(anonymous namespace)::k_fft_cols<double, 2, 1>(dnslab::FFTArgs<double>)") == "fft_z"
    assert k("void dnslab::(anonymous namespace)::k_fft_cols<float, 0, 0>(dnslab::FFTArgs<float>)") == "fft_y"
    assert k("void dnslab::(anonymous namespace)::k_fft_cols<double, 1, 2>(dnslab::FFTArgs<double>)") == "fft_y"
    assert k("void dnslab::(anonymous namespace)::k_fft_yz<double>(dnslab::FFTArgs<double>)") == "fft_yz"
    assert k("void dnslab::(anonymous namespace)::k_fft_yz<double, 8>(dnslab::FFTArgs<double>)") == "fft_yz"
    assert k("void dnslab::(anonymous namespace)::k_fft_yz_b<float, 16>(dnslab::BRec<...> const*)") == "fft_yz"
    assert k("dnslab::(anonymous namespace)::k_refine_correct(dnslab::RefineCorrArgs)") == "correct"
    assert k("dnslab::(anonymous namespace)::k_refine_res(dnslab::RefineResArgs)") == "refine_res"
    assert k("dnslab::(anonymous namespace)::k_refine_res_ib(dnslab::RefineResArgs)") == "refine_res_ib"
    assert k("void dnslab::(anonymous namespace)::k_mom_pair<double, 1>(dnslab::MomPairArgs<double>)") == "mom_pair"
    assert k("void dnslab::(anonymous namespace)::k_mom_pair_b<float, 0>(dnslab::BRec<...> const*)") == "mom_pair"
    assert k("void dnslab::(anonymous namespace)::k_sca_pair<double, 0>(dnslab::ScaPairArgs<double>)") == "scalar_pair"
    assert k("void dnslab::(anonymous namespace)::k_filter_ring<double, 3>(dnslab::FiltArgs<double>)") == "filter"
    assert k("void dnslab::(anonymous namespace)::k_filter_ring_b<float, 1>(dnslab::BRec<...> const*)") == "filter_c"
    assert k("void dnslab::(anonymous namespace)::k_correct_ring<double>(dnslab::CorrArgs<double>)") == "correct"
    assert k("dnslab::(anonymous namespace)::k_refine_correct_ring(dnslab::RefineCorrArgs)") == "correct"
    assert k("dnslab::(anonymous namespace)::k_advance(dnslab::AdvanceArgs)") is None
    assert k("__amd_rocclr_copyBuffer") is None


def write_csv(path, rows):
    cols = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w") as f:
        f.write(",".join(f'"{c}"' for c in cols) + "\n")
        for i, (name, counter, value) in enumerate(rows):
            f.write(f'{i},{i},"{name}","{counter}",{value}\n')


def test_traffic_table_calibration(tmp_path):
    mom = "void dnslab::(anonymous namespace)::k_mom_stage<double, 0, true>(dnslab::MomArgs<double>)"
    mom1 = "void dnslab::(anonymous namespace)::k_mom_stage<double, 1, true>(dnslab::MomArgs<double>)"
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    cf, cw = tmp_path / "cf.csv", tmp_path / "cw.csv"
    write_csv(f, [(mom, "FETCH_SIZE", 100.0), (mom, "FETCH_SIZE", 300.0), (mom1, "FETCH_SIZE", 600.0)])
    write_csv(w, [(mom, "WRITE_SIZE", 50.0), (mom1, "WRITE_SIZE", 150.0)])
    # a 1 GiB copy that reads back half its bytes and writes all of them
    write_csv(cf, [("__amd_rocclr_copyBuffer", "FETCH_SIZE", (1 << 30) / 1024 / 2)])
    write_csv(cw, [("__amd_rocclr_copyBuffer", "WRITE_SIZE", (1 << 30) / 1024)])
    t = bench.traffic_table(str(f), str(w), str(cf), str(cw))
    assert abs(t["fetch_scale"] - 2.0) < 1e-12 and abs(t["write_scale"] - 1.0) < 1e-12
    k = t["kernels"]["mom_stage"]
    # stage means: fetch (200 + 600) / 2 KiB x 2, write (50 + 150) / 2 KiB
    assert abs(k["fetch_bytes"] - 800 * 1024) < 1e-6
    assert abs(k["write_bytes"] - 100 * 1024) < 1e-6
    assert abs(k["bytes"] - 900 * 1024) < 1e-6


def test_step_byte_model():
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=3, seed=2204)
    kb = bench.kernel_bytes(sc, 8)
    n = sc.ncells
    assert kb["mom_stage"] == n * 97
    assert kb["div"] == n * 32
    assert kb["correct"] == n * 57
    per = bench.step_bytes(sc, 8) / n
    # half spectrum per cell: 16 B x (nx/2 + 1) / nx = 8.25 B; one solve reads and
    # writes it in each of x (with the 8 B real field), y twice and z
    solve = 2 * (8 + 8.25) + 2 * (2 * 8.25) + 2 * 8.25
    ib = bench.near_solid_cells(sc) * (4 + 1 + 24) / n
    expect = 4 * 97 + 4 * 57 + 32 + 57 + 49 + 17 + 4 * (solve + ib)
    assert abs(per - expect) < 1e-9, (per, expect)
    # the fused y/z pass reads and writes the spectrum once instead of three times
    fused = bench.step_bytes(sc, 8, fused_yz=True) / n
    assert abs(per - fused - 4 * (2 * 2 * 8.25)) < 1e-9
    assert bench.step_bytes(sc, 8, per_stage=True) > 2 * bench.step_bytes(sc, 8)
    # RK4 stages two per pass: momentum 9 + 12 instead of 48 field accesses
    # (+ one mask byte per pass), scalar 6 + 7 instead of 28
    pairs = bench.step_bytes(sc, 8, mom_pairs=True, sca_pairs=True) / n
    assert abs(per - pairs - (4 * 97 - (21 * 8 + 2)) - (4 * 57 - (13 * 8 + 2))) < 1e-9
    assert bench.step_bytes(sc, 4) < 0.6 * bench.step_bytes(sc, 8)


def test_small_room_workloads():
    """The serving-stream room sizes are bench workloads of their own: 10 m
    long rooms with 4 boxes, each with a description naming its grid."""
    for name, g in bench.SMALL_ROOMS.items():
        sc = bench.workload(name)
        assert (sc.nx, sc.ny, sc.nz) == g
        assert np.isclose(sc.spacing[0] * sc.nx, 10.0)
        assert f"{g[0]}x{g[1]}x{g[2]}" in bench.WORKLOADS[name]
