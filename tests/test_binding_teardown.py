"""The binding's exit-time teardown, on the CPU with a recording stand-in
for the library: live hierarchies are freed before their context is
destroyed, the allocator callbacks are dropped after the destroy, and a
hierarchy collected after the teardown calls nothing."""
import gc

from paper_2204_11757_amd import spc


class FakeLib:
    def __init__(self):
        self.calls = []

    def spc_hier_free(self, h):
        self.calls.append(("hier_free", h))

    def spc_destroy(self, h):
        self.calls.append(("destroy", h))
        return 0


def fake_context(tag):
    ctx = object.__new__(spc.Context)
    ctx.device = 0
    ctx.h = tag
    ctx._alloc = lambda *a: None
    ctx._free = lambda *a: None
    return ctx


def test_teardown_order(monkeypatch):
    fake = FakeLib()
    monkeypatch.setattr(spc, "lib", lambda: fake)
    monkeypatch.setattr(spc, "_contexts", {})
    monkeypatch.setattr(spc, "_live", spc.weakref.WeakSet())
    monkeypatch.setattr(spc, "_shutting_down", False)
    ctx = fake_context("ctx0")
    spc._contexts[0] = ctx
    h1 = spc.Hierarchy(ctx, "h1", 10)
    h2 = spc.Hierarchy(ctx, "h2", 10)
    h2.free()                                  # freed by the user: not freed again
    assert fake.calls == [("hier_free", "h2")]
    spc._teardown()
    assert fake.calls == [("hier_free", "h2"), ("hier_free", "h1"), ("destroy", "ctx0")]
    assert spc._shutting_down
    assert ctx.h is None and ctx._alloc is None and ctx._free is None
    assert not spc._contexts
    # a hierarchy still referenced after the teardown does nothing when collected
    h3 = spc.Hierarchy(ctx, "h3", 10)
    n = len(fake.calls)
    del h3
    gc.collect()
    assert len(fake.calls) == n
    del h1, h2


def test_free_after_context_destroyed_raises(monkeypatch):
    fake = FakeLib()
    monkeypatch.setattr(spc, "lib", lambda: fake)
    monkeypatch.setattr(spc, "_live", spc.weakref.WeakSet())
    monkeypatch.setattr(spc, "_shutting_down", False)
    ctx = fake_context(None)
    h = spc.Hierarchy(ctx, "h", 4)
    try:
        h.free()
    except RuntimeError as e:
        assert "destroyed" in str(e)
    else:
        raise AssertionError("free after the context was destroyed must raise")
    assert fake.calls == []
    h.h = None
