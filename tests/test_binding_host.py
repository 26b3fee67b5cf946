"""Host-side checks of the Python binding's object lifetimes (no GPU: the
C library is replaced by a recording stub)."""
import ctypes
import gc

import paper_1906_12018_amd as pll


class StubLib:
    def __init__(self):
        self.freed = []
        self.owned = []

    def pll_server_create(self, opts, out):
        out._obj.value = 1234
        return 0

    def pll_server_add_index(self, srv, handle, own, iid):
        self.owned.append(own)
        iid._obj.value = 7
        return 0

    def pll_index_free(self, h):
        self.freed.append(h.value if hasattr(h, "value") else h)

    def pll_server_destroy(self, srv):
        pass


def test_non_owned_index_is_released_by_python_and_retained_by_the_server(monkeypatch):
    """Without ownership the C server takes its own reference (pll.h), so the
    binding keeps no Python reference: dropping the Index drops the caller's
    reference at once, and the server still holds one."""
    stub = StubLib()
    monkeypatch.setattr(pll, "load_library", lambda *a, **k: stub)
    srv = pll.Server()
    iid = srv.add_index(pll.Index(0xABC, None))  # the caller drops its reference at once
    gc.collect()
    assert iid == 7 and stub.freed == [0xABC] and stub.owned == [0]
    srv.close()
    gc.collect()
    assert stub.freed == [0xABC]


def test_server_owned_index_is_not_freed_by_python(monkeypatch):
    stub = StubLib()
    monkeypatch.setattr(pll, "load_library", lambda *a, **k: stub)
    srv = pll.Server()
    idx = pll.Index(0xDEF, None)
    srv.add_index(idx, take_ownership=True)
    del idx
    gc.collect()
    srv.close()
    gc.collect()
    assert stub.freed == []                       # the C server frees it, not Python
