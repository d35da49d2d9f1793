"""Host logic of batching and serving: instance generators and packing."""
import numpy as np

from paper_1810_07485_amd import batching, workloads


def test_batch_instances_follow_the_stated_distribution():
    a = workloads.batch_instances()
    b = workloads.batch_instances()
    assert a == b and len(a) == 512
    L = np.array([i.L for i in a])
    beta = np.array([i.beta for i in a])
    assert (L % 2 == 0).all() and L.min() >= 64 and L.max() <= 16384
    assert (beta >= L / 4).all() and (beta <= L).all()
    assert [i.seed for i in a] == list(range(1, 513))
    # log-uniform: the median of log L sits near the middle of the range
    assert abs(np.median(np.log(L)) - 0.5 * (np.log(64) + np.log(16384))) < 0.4


def test_serving_jobs_are_a_poisson_stream():
    j = workloads.serving_jobs(400, rate=2.0)
    t = np.array([x.arrival for x in j])
    assert (np.diff(t) > 0).all()
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.5) < 0.08
    assert {x.S for x in j} == {0.5, 4.0}
    assert {x.L for x in j} == {1024, 4096, 16384}
    assert all(x.beta in (x.L / 2, float(x.L)) for x in j)
    assert {x.sweeps for x in j} == {100, 1000}
    assert [x.seed for x in j] == [1000 + i for i in range(400)]


def test_pack_first_fit_decreasing():
    sizes = [5, 9, 1, 4, 7, 3, 12]
    g = batching.pack(sizes, 10)
    assert sorted(sum(g, [])) == list(range(len(sizes)))
    for grp in g:
        tot = sum(sizes[i] for i in grp)
        assert tot <= 10 or len(grp) == 1
    # largest first: 12 alone, 9+1, 7+3, 5+4
    assert sorted(sorted(sizes[i] for i in grp) for grp in g) == [[1, 9], [3, 7], [4, 5], [12]]


def test_admission_accounting():
    from paper_1810_07485_amd.serve import Admission
    g = Admission.GROWTH
    a = Admission(100, max_resident=3)
    assert a.fits_ever(100) and not a.fits_ever(101)
    assert a.fits_ever(0, 100 / g) and not a.fits_ever(1, 100 / g)
    assert a.try_admit(60) and not a.try_admit(50) and a.try_admit(40)
    assert a.used == 100 and a.resident == 2
    a.release(60)
    assert a.try_admit(30) and a.try_admit(1) and not a.try_admit(1)  # slot limit
    assert a.resident == 3 and a.used == 71
    # scratch counts with the arena's growth headroom, and the arena's
    # current size bounds it from below (it does not shrink)
    b = Admission(100)
    assert b.try_admit(10, 40)                  # 10 + 1.33 * 40 = 63
    assert not b.try_admit(10, 25)              # 20 + 1.33 * 65 = 106 > 100
    assert b.try_admit(5, 10)                   # 15 + 1.33 * 50 = 81
    b.release(10, 40)
    assert b.state == 5 and b.scratch == 10
    assert not b.try_admit(10, 1, arena_bytes=90)  # 15 + max(90, ...) > 100
    assert b.try_admit(10, 1, arena_bytes=60)
