"""Per-solve history (sgtt_solve_history): one record per outer FGMRES
iteration and one per refinement cycle, consistent with the solve's stats."""
import pytest

from synthetic_inputs import CONFIGS

pytestmark = pytest.mark.gpu


def test_solve_history_matches_stats():
    from paper_1906_06785_amd import sgtt as sg
    print("solve history c1", flush=True)
    ctx = sg.Context(0)
    S = sg.System(ctx, CONFIGS["C1"])
    x, st, rc = S.solve(S.rhs(), S.pair(64, 1024), restart=20, relax=1)
    assert rc == 0
    h = S.history()
    its = [r for r in h if r["iter"] > 0]
    ends = [r for r in h if r["iter"] == -1]
    assert len(its) == st["outer_iters"] and len(ends) == st["cycles"]
    assert ends[-1]["rel"] == st["rel_residual"]
    assert tuple(ends[-1]["rank_z_u"]) == x.ranks[0] and tuple(ends[-1]["rank_z_p"]) == x.ranks[1]
    assert max(r["rank_v_u"][1] for r in its) == st["max_rank_krylov_u"]
    # within a cycle the iterations count up and the correction system's
    # residual ends below where it started; the cycle ends' exact residuals
    # fall, the last one to the solve's tolerance
    for c in range(st["cycles"]):
        rs = [r for r in its if r["cycle"] == c]
        assert [r["iter"] for r in rs] == list(range(1, len(rs) + 1))
        assert rs[-1]["rel"] < rs[0]["rel"] or len(rs) == 1
    assert all(ends[i + 1]["rel"] < ends[i]["rel"] for i in range(len(ends) - 1))
    assert ends[-1]["rel"] <= 1e-8
    assert all(h[i]["seconds"] <= h[i + 1]["seconds"] for i in range(len(h) - 1))
    # a later solve replaces the history
    S.solve(S.rhs(), S.pair(64, 1024), restart=20, relax=1, max_cycles=1, tol=1e-3)
    assert len([r for r in S.history() if r["iter"] == -1]) == 1
