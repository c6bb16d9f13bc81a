"""Stream ordering of the Python binding (host logic, no GPU): library memory is
taken on the library's stream, and a device readout into a tensor from the
caller's stream is ordered after the caller's earlier work and before its
later work.  A stand-in for torch records the calls."""
import contextlib
import ctypes as C

import paper_2601_18443_amd as P


class _Stream:
    def __init__(self, name, log):
        self.name, self.log = name, log

    def wait_stream(self, other):
        self.log.append(("wait", self.name, other.name))


class _Tensor:
    _next = 4096

    def __init__(self, shape):
        self.shape = shape
        _Tensor._next += 4096
        self.ptr = _Tensor._next

    def data_ptr(self):
        return self.ptr

    def numel(self):
        n = 1
        for s in (self.shape if isinstance(self.shape, tuple) else (self.shape,)):
            n *= s
        return n


class _Cuda:
    def __init__(self, log):
        self.log = log
        self.current = _Stream("caller", log)
        self.active = "caller"

    def current_stream(self, device=None):
        return self.current

    @contextlib.contextmanager
    def stream(self, s):
        prev, self.active = self.active, s.name
        try:
            yield
        finally:
            self.active = prev


class _Torch:
    uint8, float64 = "u8", "f64"

    def __init__(self, log):
        self.log = log
        self.cuda = _Cuda(log)

    def empty(self, shape, dtype=None, device=None):
        self.log.append(("empty", self.cuda.active))
        return _Tensor(shape)


def test_library_memory_comes_from_the_library_stream():
    log = []
    torch = _Torch(log)
    lib_stream = _Stream("library", log)
    alloc = P._TorchAllocator("cuda:0", lib_stream, torch_module=torch)
    ptr = alloc._alloc(1 << 20, None)
    assert ptr and ptr in alloc.live
    assert log == [("empty", "library")]
    alloc._free(ptr, None)
    assert ptr not in alloc.live


def test_device_readout_is_ordered_on_both_streams(monkeypatch):
    log = []
    torch = _Torch(log)

    class _Lib:
        def lbr_read_field_device(self, h, level, which, ptr, n):
            log.append(("read", level, which, n))
            return 0

    monkeypatch.setattr(P, "lib", lambda: _Lib())
    s = object.__new__(P.Solver)
    s.h = C.c_void_p(1)
    s.device = "cuda:0"
    s.torch_stream = _Stream("library", log)
    s.level_info = lambda level: {"nx": 5, "ny": 3}
    out = s.field_device(2, P.FIELD_UX, torch_module=torch)
    assert out.shape == (3, 5)
    assert log == [("empty", "caller"), ("wait", "library", "caller"), ("read", 2, P.FIELD_UX, 15),
                   ("wait", "caller", "library")]
