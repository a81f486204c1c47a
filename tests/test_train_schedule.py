"""The progressive training schedule (Sec. 5.8) as a host state machine:
doubling iterations, a new iteration only while less than half of the
training budget is used, training ended at its share of the budget.  Runs
on the CPU (no device call)."""
import pytest


@pytest.fixture(scope="module")
def M():
    import paper_2311_12818_amd as M
    M.lib()
    return M


def simulate(M, budget, frac, base, batch, per_sample):
    plan = M.mpg_train_plan(budget, frac, base)
    st = M.train_init(plan)
    t = 0.0
    events = []
    gathered = 0
    while st.phase == M.TRAIN:
        t += batch * per_sample
        gathered += batch
        it = st.iteration
        M.train_step(plan, st, batch, t)
        if st.refit:
            events.append((it, gathered, round(t, 9), st.phase))
            gathered = 0
    return events


def test_doubling_iterations_then_one_long_last_iteration(M):
    # 100 time units, 30% training (30), half of it 15; 100 samples per unit
    # of 0.01; batches of 50.  Iterations of 100, 200, 400 samples end at
    # t = 1, 3, 7 and each starts a doubled one; the 800-sample iteration is
    # complete at t = 15, when half the training budget is used, so it goes
    # on until training stops at t = 30 with 2300 samples.
    ev = simulate(M, 100.0, 0.3, 100, 50, 0.01)
    assert ev == [(0, 100, 1.0, M.TRAIN), (1, 200, 3.0, M.TRAIN), (2, 400, 7.0, M.TRAIN), (3, 2300, 30.0, M.RENDER)]


def test_training_stops_inside_an_iteration(M):
    # training share 5 (half: 2.5): iteration 0 ends at t = 1 and starts
    # iteration 1, which reaches its 200 samples at t = 3, past half the
    # training budget, so it keeps gathering until training stops at t = 5
    ev = simulate(M, 100.0, 0.05, 100, 50, 0.01)
    assert ev == [(0, 100, 1.0, M.TRAIN), (1, 400, 5.0, M.RENDER)]


def test_no_training_and_bad_plans(M):
    st = M.train_init(M.mpg_train_plan(10.0, 0.0, 100))
    assert st.phase == M.RENDER
    for plan in [M.mpg_train_plan(0.0, 0.3, 100), M.mpg_train_plan(10.0, 1.5, 100), M.mpg_train_plan(10.0, 0.3, 0)]:
        with pytest.raises(M.MPGError):
            M.train_init(plan)
