"""The read-back path that returns pivot counts, ranks, flags and norms to
the host during a solve (t2s2_debug_readback): every byte equal to a device
copy of the same buffer, for sizes around the 4-byte word and the 64 KiB
mailbox limit (beyond it the runtime's copy), misaligned starts, and reads
from 8 host threads on their own streams at once, each read following a
fresh device-side fill of its buffer (the reads of concurrent solves)."""
import ctypes as C
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import paper_2506_04732_amd as t2s2  # noqa: E402
from paper_2506_04732_amd import _lib  # noqa: E402


def _read(dev_ptr, nbytes, stream):
    out = np.empty(max(nbytes, 1), dtype=np.uint8)
    t2s2.check(_lib.lib().t2s2_debug_readback(C.c_void_p(dev_ptr), out.ctypes.data_as(C.c_void_p), nbytes,
                                              C.c_void_p(stream)))
    return out[:nbytes]


@pytest.mark.parametrize("nbytes", [0, 1, 3, 4, 5, 8, 31, 33, 1000, 4096, 65535, 65536, 65537, 200001])
@pytest.mark.parametrize("offset", [0, 1, 3])
def test_readback_bytes_exact(nbytes, offset):
    print("[case] readback", nbytes, "offset", offset, flush=True)
    g = torch.Generator(device="cpu").manual_seed(nbytes * 7 + offset)
    host = torch.randint(0, 256, (nbytes + offset + 8,), dtype=torch.uint8, generator=g)
    dev = host.cuda()
    stream = torch.cuda.current_stream().cuda_stream
    got = _read(dev.data_ptr() + offset, nbytes, stream)
    assert np.array_equal(got, host.numpy()[offset:offset + nbytes])


def test_readback_concurrent_threads():
    print("[case] readback 8 threads x 300 reads", flush=True)
    errors = []

    def worker(t):
        try:
            s = torch.cuda.Stream()
            rng = np.random.default_rng(100 + t)
            buf = torch.empty(70000, dtype=torch.int32, device="cuda")
            with torch.cuda.stream(s):
                for it in range(300):
                    val = int(rng.integers(1, 2 ** 30))
                    n = int(rng.choice([1, 2, 3, 17, 257, 4000, 16384]))
                    buf[:n].fill_(val)  # queued on s just before the read
                    got = _read(buf.data_ptr(), 4 * n, s.cuda_stream).view(np.int32)
                    if not np.all(got == val):
                        errors.append((t, it, n, val, int(got[got != val][0])))
                        return
        except Exception as e:  # report, do not hang the other threads
            errors.append((t, repr(e)))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(8)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors[:4]
