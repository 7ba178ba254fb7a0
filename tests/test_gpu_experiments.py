"""The synthetic analogue of the paper's simulation study (Figs. 4 and 5)
reproduces the paper's qualitative findings on data simulated with the full
expanded model (148 px, 32 coils compressed to 16, SNR 20):

* the expanded model reconstructs better than the partial one (no 2nd-order
  terms), with a gap that shrinks as acceleration shortens the readout;
* CS with the expanded model has the lowest NRMSE at every acceleration;
* CS (100 FISTA iterations) costs several times the LS time (20 CG
  iterations), the paper's 5-10x.
The solvers themselves are parity-tested against the oracle elsewhere."""
import pytest

pytestmark = pytest.mark.gpu


def test_expanded_model_and_cs_win():
    from paper_2211_07532_amd import experiments as ex
    res = ex.run([ex.Setting(2, 16, 20.0), ex.Setting(4, 16, 20.0)], models=("expanded", "partial"))
    e = {(r["accel"], r["model"], r["method"]): r for r in res}
    for a in (2, 4):
        for m in ("LS", "CS"):
            assert e[(a, "expanded", m)]["nrmse"] < e[(a, "partial", m)]["nrmse"]
        best = min(r["nrmse"] for r in res if r["accel"] == a)
        assert e[(a, "expanded", "CS")]["nrmse"] == best
        assert e[(a, "expanded", "CS")]["seconds"] > 2.0 * e[(a, "expanded", "LS")]["seconds"]
    gap = {a: e[(a, "partial", "LS")]["nrmse"] - e[(a, "expanded", "LS")]["nrmse"] for a in (2, 4)}
    print(f"[case] partial - expanded (LS): R=2 {gap[2]:.4f}  R=4 {gap[4]:.4f}", flush=True)
    assert gap[2] > gap[4] > 0
