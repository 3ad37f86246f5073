"""CPU checks of the replanning server's host logic (no GPU)."""

from paper_1705_02403_amd import gmt, server


class FakeRoadmap:
    def __init__(self, key, size):
        self.key, self.size, self.freed = key, size, False

    def free(self):
        self.freed = True


def make_cache(budget):
    built = []

    def build(key):
        rm = FakeRoadmap(key, 100)
        built.append(rm)
        return rm

    return server.RoadmapCache(budget, build, size_of=lambda rm: rm.size), built


def test_lru_evicts_least_recent_unpinned():
    c, built = make_cache(250)
    a = c.acquire("a")
    c.release("a")
    b = c.acquire("b")
    c.release("b")
    assert c.acquire("a") is a  # hit refreshes a
    c.release("a")
    c.acquire("c")  # needs room: evicts b (least recent)
    c.release("c")
    assert built[1].freed and not built[0].freed
    assert c.hits == 1 and c.misses == 3 and c.evictions == 1 and c.bytes == 200


def test_pinned_roadmaps_are_not_evicted():
    c, built = make_cache(150)
    c.acquire("a")  # pinned
    c.acquire("b")  # over budget, but a is pinned: both stay
    assert not built[0].freed and c.bytes == 200
    c.release("a")
    c.release("b")
    c.acquire("c")
    assert built[0].freed  # a now unpinned and least recent


def test_roadmap_bytes_formula():
    e = server.roadmap_bytes(100, 2, gmt.GMT_COST_EUCLIDEAN, 1000)
    ec = server.roadmap_bytes(100, 2, gmt.GMT_COST_EUCLIDEAN, 1000, cap=16)
    d = server.roadmap_bytes(100, 6, gmt.GMT_COST_DOUBLE_INTEGRATOR, 1000)
    assert e == 4 * 200 + 404 + 400 + 8 * (1000 + 256)
    assert ec == 4 * 200 + 404 + 400 + 8 * (1600 + 256)
    assert d == 4 * 600 + 404 + 4000 + 12 * (1000 + 256) + 8000 + 404 + 4000 + 3200
