"""Python API over the C-ABI.  PyTorch provides device memory and streams only.

>>> ctx = Context(0)
>>> c = ctx.mul(a, Na, b, Nb)      # a: (da, ceil(Na/64)) int64 CUDA tensor, ...
"""
from __future__ import annotations

import ctypes

import torch

from . import _native as nat


def out_bits(da: int, Na: int, db: int, Nb: int) -> int:
    return int(nat.zpm_out_bits(da, Na, db, Nb))


def out_words(da: int, Na: int, db: int, Nb: int) -> int:
    return (out_bits(da, Na, db, Nb) + 63) // 64


def plan(da: int, Na: int, db: int, Nb: int, K: int = 0, np: int = 0) -> dict:
    info = nat.PlanInfo()
    nat.check(nat.zpm_plan(da, Na, db, Nb, K, np, ctypes.byref(info)), "zpm_plan")
    return info.as_dict()


def kronecker_plan(da: int, Na: int, db: int, Nb: int, chunk_bits: int = 0) -> dict:
    """The Kronecker reshaping zpm_mul_kronecker would use (host only)."""
    info = nat.KronInfo()
    nat.check(nat.zpm_kronecker_plan(da, Na, db, Nb, chunk_bits, ctypes.byref(info)),
              "zpm_kronecker_plan")
    return info.as_dict()


KERNEL_KINDS = ["bivariate_representation", "col_pass_fwd", "convolve_rows", "col_pass_inv",
                "recovering_product", "batch", "p64_convert_in", "p64_y_fwd", "p64_x_convolve",
                "p64_y_inv", "p64_recover", "gfp_convert_in", "gfp_y_fwd", "gfp_x_convolve",
                "gfp_y_inv", "gfp_recover"]


def plan_p64(da: int, Na: int, db: int, Nb: int, K: int = 0, np: int = 0) -> dict:
    """Plan of the 64-bit prime variant (host only); K, np: 0 = choose."""
    info = nat.P64Info()
    nat.check(nat.zpm_plan_p64(da, Na, db, Nb, K, np, ctypes.byref(info)), "zpm_plan_p64")
    return info.as_dict()


def plan_gfp(da: int, Na: int, db: int, Nb: int, K: int = 0, k: int = 0) -> dict:
    """Plan of the generalized Fermat prime variant (host only); K, k: 0 = choose."""
    info = nat.GfpInfo()
    nat.check(nat.zpm_plan_gfp(da, Na, db, Nb, K, k, ctypes.byref(info)), "zpm_plan_gfp")
    return info.as_dict()


def gfp_prime(k: int) -> tuple[int, int]:
    """Radix r and bit length of the generalized Fermat prime r^k + 1 of k digits."""
    r, lp = ctypes.c_int32(), ctypes.c_int32()
    nat.check(nat.zpm_gfp_prime(k, ctypes.byref(r), ctypes.byref(lp)), "zpm_gfp_prime")
    return r.value, lp.value


def gfp_root(k: int, log2_L: int) -> list[int]:
    """Balanced radix-r digits of the order-2^log2_L root the y-transforms use."""
    buf = (ctypes.c_int32 * k)()
    nat.check(nat.zpm_gfp_root(k, log2_L, buf), "zpm_gfp_root")
    return list(buf)


def prime64(k: int) -> tuple[int, int]:
    """The k-th 64-bit prime (largest first) and a primitive 2^21-th root of unity."""
    p, r = ctypes.c_uint64(), ctypes.c_uint64()
    nat.check(nat.zpm_prime64(k, ctypes.byref(p), ctypes.byref(r)), "zpm_prime64")
    return p.value, r.value


def device_limits(device: int = 0) -> dict:
    ncu, lb, lc = nat.c_i32(), nat.c_i64(), nat.c_i64()
    nat.check(nat.zpm_device_limits(device, ctypes.byref(ncu), ctypes.byref(lb), ctypes.byref(lc)),
              "zpm_device_limits")
    return {"cus": ncu.value, "lds_per_block": lb.value, "lds_per_cu": lc.value}


def prime(k: int) -> tuple[int, int]:
    p, r = nat.c_u32(), nat.c_u32()
    nat.check(nat.zpm_prime(k, ctypes.byref(p), ctypes.byref(r)), "zpm_prime")
    return p.value, r.value


def from_ints(values, N: int | None = None, device="cuda") -> tuple[torch.Tensor, int]:
    """Python ints -> (d, ceil(N/64)) int64 tensor of N-bit two's complement words, N.

    N defaults to the smallest width that holds every value (at least 2)."""
    vals = [int(v) for v in values]
    if N is None:
        N = max([2] + [v.bit_length() + 1 for v in vals])
    lo, hi = -(1 << (N - 1)), (1 << (N - 1)) - 1
    w = (N + 63) // 64
    buf = bytearray()
    for v in vals:
        if not lo <= v <= hi:
            raise ValueError(f"{v} does not fit in {N}-bit two's complement")
        buf += v.to_bytes(8 * w, "little", signed=True)
    t = torch.frombuffer(buf, dtype=torch.int64).clone() if vals else torch.empty(0, dtype=torch.int64)
    return t.reshape(len(vals), w).to(device), N


def to_ints(t: torch.Tensor) -> list[int]:
    """(d, w) int64 tensor of two's complement words -> Python ints."""
    raw = t.detach().cpu().contiguous().numpy().tobytes()
    w = t.shape[1] if t.dim() == 2 else 1
    return [int.from_bytes(raw[8 * w * i: 8 * w * (i + 1)], "little", signed=True)
            for i in range(t.shape[0])]


# torch's current stream as a raw handle without building a Stream object (a few
# microseconds per call, which small products notice); the public route otherwise
_current_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream_handle(stream) -> int | None:
    if stream is None:
        if _current_raw_stream is not None:
            return _current_raw_stream(torch.cuda.current_device())
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check_operand(t: torch.Tensor, N: int, name: str) -> int:
    if t.dtype != torch.int64 or not t.is_cuda or t.dim() != 2:
        raise ValueError(f"{name} must be a 2-D int64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.shape[1] != (N + 63) // 64:
        raise ValueError(f"{name} has {t.shape[1]} words per coefficient, N={N} needs {(N + 63) // 64}")
    return t.shape[0]


class Context:
    """A zpm context on one device (tables, plan constants and workspace)."""

    def __init__(self, device: int = 0):
        self.device = device
        h = nat.c_vp()
        nat.check(nat.zpm_create(ctypes.byref(h), device), "zpm_create")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            nat.zpm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def reserve(self, workspace_bytes: int, max_len: int, max_bits: int, max_plans: int = 0) -> None:
        """Fix tables, workspace and plan slots (zpm_reserve): later products of at most
        these sizes allocate nothing and never wait for the device."""
        nat.check(nat.zpm_reserve(self._h, workspace_bytes, max_len, max_bits, max_plans),
                  "zpm_reserve")

    def set_check_inputs(self, on: bool) -> None:
        """Checked-input mode (ZPM_OPT_CHECK_INPUTS): products fail with ZPM_ERANGE when an
        input coefficient has bits at or above N that are not sign copies."""
        nat.check(nat.zpm_set_option(self._h, nat.ZPM_OPT_CHECK_INPUTS, 1 if on else 0),
                  "zpm_set_option")

    def mul(self, a: torch.Tensor, Na: int, b: torch.Tensor, Nb: int, wc: int | None = None,
            out: torch.Tensor | None = None, stream=None, K: int = 0, np: int = 0) -> torch.Tensor:
        """Exact product: (da+db-1, wc) int64 tensor of two's complement words."""
        da = _check_operand(a, Na, "a")
        db = _check_operand(b, Nb, "b")
        need = out_words(da, Na, db, Nb) if (da and db) else 1
        wc = need if wc is None else wc
        n = da + db - 1 if (da and db) else 0
        if out is None:
            out = torch.empty((n, wc), dtype=torch.int64, device=a.device)
        elif out.shape != (n, wc) or out.dtype != torch.int64 or not out.is_contiguous():
            raise ValueError("out has the wrong shape or dtype")
        st = _stream_handle(stream)
        if K or np:
            rc = nat.zpm_mul_ex(self._h, a.data_ptr(), da, Na, b.data_ptr(), db, Nb,
                                out.data_ptr() if n else None, wc, K, np, 0, None, st)
        else:
            rc = nat.zpm_mul(self._h, a.data_ptr(), da, Na, b.data_ptr(), db, Nb,
                             out.data_ptr() if n else None, wc, st)
        nat.check(rc, "zpm_mul")
        return out

    def mul_noalloc(self, a: torch.Tensor, Na: int, b: torch.Tensor, Nb: int,
                    out: torch.Tensor, stream=None) -> torch.Tensor:
        """c = a * b into the caller's `out` with the library's fixed scratch array as the
        workspace (zpm_mul_noalloc): nothing is allocated.  The context's tables must cover
        the sizes (zpm_reserve, or an earlier product of the same sizes)."""
        da = _check_operand(a, Na, "a")
        db = _check_operand(b, Nb, "b")
        n = da + db - 1 if (da and db) else 0
        if n and (out.dim() != 2 or out.shape[0] != n or out.dtype != torch.int64
                  or not out.is_contiguous()):
            raise ValueError("out has the wrong shape or dtype")
        nat.check(nat.zpm_mul_noalloc(self._h, a.data_ptr(), da, Na, b.data_ptr(), db, Nb,
                                      out.data_ptr() if n else None, out.shape[1] if n else 1,
                                      _stream_handle(stream)), "zpm_mul_noalloc")
        return out

    def mul_kronecker(self, a: torch.Tensor, Na: int, b: torch.Tensor, Nb: int,
                      chunk_bits: int = 0, out: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
        """c = a * b through Kronecker reshaping (chunks of chunk_bits, 0 = choose)."""
        da = _check_operand(a, Na, "a")
        db = _check_operand(b, Nb, "b")
        n = da + db - 1 if (da and db) else 0
        wc = out_words(da, Na, db, Nb) if n else 1
        if out is None:
            out = torch.empty((n, wc), dtype=torch.int64, device=a.device)
        nat.check(nat.zpm_mul_kronecker(self._h, a.data_ptr(), da, Na, b.data_ptr(), db, Nb,
                                        out.data_ptr() if n else None, out.shape[1] if n else wc,
                                        chunk_bits, _stream_handle(stream)), "zpm_mul_kronecker")
        return out

    def mul_p64(self, a: torch.Tensor, Na: int, b: torch.Tensor, Nb: int, K: int = 0, np: int = 0,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """c = a * b with one to three 64-bit primes (zpm_mul_p64); K, np: 0 = choose."""
        da = _check_operand(a, Na, "a")
        db = _check_operand(b, Nb, "b")
        n = da + db - 1 if (da and db) else 0
        wc = out_words(da, Na, db, Nb) if n else 1
        if out is None:
            out = torch.empty((n, wc), dtype=torch.int64, device=a.device)
        elif out.shape != (n, wc) or out.dtype != torch.int64 or not out.is_contiguous():
            raise ValueError("out has the wrong shape or dtype")
        nat.check(nat.zpm_mul_p64(self._h, a.data_ptr(), da, Na, b.data_ptr(), db, Nb,
                                  out.data_ptr() if n else None, wc, K, np, _stream_handle(stream)),
                  "zpm_mul_p64")
        return out

    def mul_gfp(self, a: torch.Tensor, Na: int, b: torch.Tensor, Nb: int, K: int = 0, k: int = 0,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """c = a * b with one generalized Fermat prime (zpm_mul_gfp); K, k: 0 = choose."""
        da = _check_operand(a, Na, "a")
        db = _check_operand(b, Nb, "b")
        n = da + db - 1 if (da and db) else 0
        wc = out_words(da, Na, db, Nb) if n else 1
        if out is None:
            out = torch.empty((n, wc), dtype=torch.int64, device=a.device)
        elif out.shape != (n, wc) or out.dtype != torch.int64 or not out.is_contiguous():
            raise ValueError("out has the wrong shape or dtype")
        nat.check(nat.zpm_mul_gfp(self._h, a.data_ptr(), da, Na, b.data_ptr(), db, Nb,
                                  out.data_ptr() if n else None, wc, K, k, _stream_handle(stream)),
                  "zpm_mul_gfp")
        return out

    def mul_stage(self, a: torch.Tensor, Na: int, b: torch.Tensor, Nb: int, stop_after: int,
                  K: int = 0, np: int = 0, stream=None) -> tuple[torch.Tensor, dict]:
        """Run the product up to a stage and return the workspace (np, 2K, L) uint32 as int64."""
        da = _check_operand(a, Na, "a")
        db = _check_operand(b, Nb, "b")
        info = plan(da, Na, db, Nb, K, np)
        ws = torch.empty(info["workspace_bytes"] // 4, dtype=torch.int32, device=a.device)
        wc = out_words(da, Na, db, Nb)
        out = torch.empty((da + db - 1, wc), dtype=torch.int64, device=a.device)
        rc = nat.zpm_mul_ex(self._h, a.data_ptr(), da, Na, b.data_ptr(), db, Nb, out.data_ptr(), wc,
                            info["K"], info["np"], stop_after, ws.data_ptr(), _stream_handle(stream))
        nat.check(rc, "zpm_mul_ex")
        L = 1 << info["log2_L"]
        w = ws.to(torch.int64) & 0xFFFFFFFF
        return w.view(info["np"], 2 * info["K"], L), info

    def mul_batch(self, items, graph: bool = False, K: int = 0, stream=None, outs=None,
                  persistent: bool = False):
        """Products of many (a, Na, b, Nb) in one call (grouped launches per level, or with
        ``persistent`` all of them in one persistent launch, which waits for the device).

        items: list of (a, Na, b, Nb) with a, b int64 CUDA tensors as for mul.
        Returns the list of output tensors (allocated unless ``outs`` is given).
        The library copies the Job array during the call; the last one is kept on the
        context only for inspection.
        """
        n = len(items)
        jobs = (nat.Job * max(n, 1))()
        res = []
        for i, (a, Na, b, Nb) in enumerate(items):
            da = _check_operand(a, Na, "a")
            db = _check_operand(b, Nb, "b")
            nout = da + db - 1 if (da and db) else 0
            wc = out_words(da, Na, db, Nb) if nout else 1
            o = outs[i] if outs is not None else torch.empty((nout, wc), dtype=torch.int64,
                                                            device=a.device)
            if outs is not None:
                wc = o.shape[1] if o.dim() == 2 else wc
            res.append(o)
            jobs[i].a, jobs[i].da, jobs[i].Na = a.data_ptr(), da, Na
            jobs[i].b, jobs[i].db, jobs[i].Nb = b.data_ptr(), db, Nb
            jobs[i].c, jobs[i].wc = (o.data_ptr() if nout else None), wc
        self._batch_jobs = jobs
        flags = (nat.ZPM_BATCH_GRAPH if graph else 0) | (nat.ZPM_BATCH_PERSISTENT if persistent else 0)
        st = _stream_handle(stream)
        if K:
            rc = nat.zpm_mul_batch_ex(self._h, jobs, n, flags, K, st)
        else:
            rc = nat.zpm_mul_batch(self._h, jobs, n, flags, st)
        nat.check(rc, "zpm_mul_batch")
        return res

    def mul_operand_batch(self, items, graph: bool = False, stream=None, outs=None):
        """Products a * b for many (a, Na, operand) in one call (zpm_mul_operand_batch):
        each operand's b is taken as its resident spectra.  Returns the output tensors."""
        n = len(items)
        jobs = (nat.OperandJob * max(n, 1))()
        res = []
        for i, (a, Na, op) in enumerate(items):
            jobs[i], o = op.job(a, Na, outs[i] if outs is not None else None)
            res.append(o)
        self._batch_jobs = (jobs, [op for (_, _, op) in items])
        flags = nat.ZPM_BATCH_GRAPH if graph else 0
        nat.check(nat.zpm_mul_operand_batch(self._h, jobs, n, flags, _stream_handle(stream)),
                  "zpm_mul_operand_batch")
        return res

    def _jobs(self, items, outs=None):
        n = len(items)
        jobs = (nat.Job * max(n, 1))()
        res = []
        for i, (a, Na, b, Nb) in enumerate(items):
            da = _check_operand(a, Na, "a")
            db = _check_operand(b, Nb, "b")
            nout = da + db - 1 if (da and db) else 0
            wc = out_words(da, Na, db, Nb) if nout else 1
            o = outs[i] if outs is not None else None
            res.append(o)
            jobs[i].a, jobs[i].da, jobs[i].Na = a.data_ptr(), da, Na
            jobs[i].b, jobs[i].db, jobs[i].Nb = b.data_ptr(), db, Nb
            jobs[i].c, jobs[i].wc = (o.data_ptr() if (o is not None and nout) else None), \
                (o.shape[1] if o is not None and o.dim() == 2 else wc)
        return jobs, res

    def tune(self, items, cache_path: str | None = None, stream=None) -> dict:
        """Autotune (K, column tile) per size class on a sample of (a, Na, b, Nb);
        returns {class: (K, T)}."""
        jobs, _ = self._jobs(items)
        path = cache_path.encode() if cache_path else None
        nat.check(nat.zpm_tune(self._h, jobs, len(items), path, _stream_handle(stream)), "zpm_tune")
        return self.tune_table()

    def tune_load(self, cache_path: str) -> None:
        nat.check(nat.zpm_tune_load(self._h, cache_path.encode()), "zpm_tune_load")

    def tune_table(self) -> dict:
        """{size class: (K, column tile)} chosen by tune or loaded by tune_load."""
        n = nat.c_i32()
        nat.check(nat.zpm_tune_get(self._h, None, None, None, 0, ctypes.byref(n)), "zpm_tune_get")
        cl = (nat.c_i32 * max(n.value, 1))()
        ks = (nat.c_i32 * max(n.value, 1))()
        ts = (nat.c_i32 * max(n.value, 1))()
        nat.check(nat.zpm_tune_get(self._h, cl, ks, ts, n.value, ctypes.byref(n)), "zpm_tune_get")
        return {cl[i]: (ks[i], ts[i]) for i in range(n.value)}

    def profile_begin(self, kinds=None) -> None:
        """Start per-kernel timing, of every kernel or only of the named kinds."""
        if kinds is None:
            nat.check(nat.zpm_profile_begin(self._h), "zpm_profile_begin")
        else:
            mask = 0
            for k in kinds:
                mask |= 1 << KERNEL_KINDS.index(k)
            nat.check(nat.zpm_profile_begin_kinds(self._h, mask), "zpm_profile_begin_kinds")

    def profile_end(self) -> dict:
        """{kernel name: (launches, total GPU ms)} since profile_begin."""
        buf = (nat.KernelTime * 32)()
        n = nat.c_i32()
        nat.check(nat.zpm_profile_end(self._h, buf, 32, ctypes.byref(n)), "zpm_profile_end")
        return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(min(n.value, 32))}

    def sync(self, stream=None) -> None:
        nat.check(nat.zpm_sync(self._h, _stream_handle(stream)), "zpm_sync")


class Operand:
    """A factor b transformed once (zpm_operand_*), for products a * b with any a of
    at most da_max coefficients and Na_max bits.  Keeps a reference to b."""

    def __init__(self, ctx: Context, b: torch.Tensor, Nb: int, da_max: int, Na_max: int,
                 K: int = 0, stream=None):
        db = _check_operand(b, Nb, "b")
        h = nat.c_vp()
        nat.check(nat.zpm_operand_create(ctx.handle, b.data_ptr(), db, Nb, da_max, Na_max, K,
                                         ctypes.byref(h), _stream_handle(stream)),
                  "zpm_operand_create")
        self._h, self._ctx, self._b = h, ctx, b
        self.db, self.Nb = db, Nb

    def info(self) -> dict:
        info = nat.PlanInfo()
        nat.check(nat.zpm_operand_info(self._h, ctypes.byref(info)), "zpm_operand_info")
        return info.as_dict()

    def mul(self, a: torch.Tensor, Na: int, out: torch.Tensor | None = None,
            stream=None) -> torch.Tensor:
        """c = a * b as a (da + db - 1, wc) int64 tensor."""
        da = _check_operand(a, Na, "a")
        n = da + self.db - 1 if da else 0
        wc = out_words(da, Na, self.db, self.Nb) if n else 1
        if out is None:
            out = torch.empty((n, wc), dtype=torch.int64, device=a.device)
        nat.check(nat.zpm_mul_operand(self._ctx.handle, a.data_ptr(), da, Na, self._h,
                                      out.data_ptr() if n else None, out.shape[1] if n else wc,
                                      _stream_handle(stream)), "zpm_mul_operand")
        return out

    def job(self, a: torch.Tensor, Na: int, out: torch.Tensor | None = None):
        """(zpm_operand_job for a * b, output tensor); the job holds raw pointers, so the
        caller keeps a, out and this operand alive while it is in use."""
        da = _check_operand(a, Na, "a")
        n = da + self.db - 1 if da else 0
        wc = out_words(da, Na, self.db, self.Nb) if n else 1
        if out is None:
            out = torch.empty((n, wc), dtype=torch.int64, device=a.device)
        elif out.dim() != 2 or out.shape[0] != n or out.dtype != torch.int64 or not out.is_contiguous():
            raise ValueError("out has the wrong shape or dtype")
        j = nat.OperandJob()
        j.a, j.da, j.Na, j.op = a.data_ptr(), da, Na, self._h
        j.c, j.wc = (out.data_ptr() if n else None), (out.shape[1] if n else wc)
        return j, out

    def close(self) -> None:
        if getattr(self, "_h", None):
            nat.zpm_operand_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over a context (see zpm_server_* in include/zpm.h).

    ``submit`` takes CUDA tensors as ``Context.mul`` does and keeps references to them
    until the request is reported finished, so the caller need not.  Results arrive
    in the output tensor given to (or returned by) ``submit``.
    """

    def __init__(self, ctx: Context | None, hbm_budget: int = 0, n_streams: int = 0,
                 max_batch: int = 0, large_bits: float = 0.0, single_product: bool = False,
                 large_streams: int = 0, simulate: dict | None = None, min_batch: int = 0,
                 linger_s: float = 0.0):
        cfg = nat.ServerConfig(hbm_budget, n_streams, max_batch, large_bits, int(single_product),
                               large_streams, min_batch, linger_s)
        h = nat.c_vp()
        if simulate is not None:
            rc = nat.zpm_server_create_simulated(ctypes.byref(cfg), simulate["bits_per_s"],
                                                 simulate.get("overhead_s", 0.0),
                                                 simulate.get("fail_after", -1), ctypes.byref(h))
        else:
            rc = nat.zpm_server_create_ex(ctx.handle, ctypes.byref(cfg), ctypes.byref(h))
        nat.check(rc, "zpm_server_create")
        self._h = h
        self._ctx = ctx
        self._keep: dict[int, tuple] = {}

    def close(self) -> None:
        if getattr(self, "_h", None):
            nat.zpm_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit_job(self, job: nat.Job, keep=()) -> int:
        t = nat.c_u64()
        nat.check(nat.zpm_server_submit(self._h, ctypes.byref(job), ctypes.byref(t)),
                  "zpm_server_submit")
        if keep:
            self._keep[t.value] = tuple(keep)
        return t.value

    def submit(self, a: torch.Tensor, Na: int, b: torch.Tensor, Nb: int,
               out: torch.Tensor | None = None) -> tuple[int, torch.Tensor]:
        """Queue a * b; returns (ticket, output tensor)."""
        da = _check_operand(a, Na, "a")
        db = _check_operand(b, Nb, "b")
        n = da + db - 1 if (da and db) else 0
        wc = out_words(da, Na, db, Nb) if n else 1
        if out is None:
            out = torch.empty((n, wc), dtype=torch.int64, device=a.device)
        elif out.dim() != 2 or out.shape[0] != n or out.dtype != torch.int64 or not out.is_contiguous():
            raise ValueError("out has the wrong shape or dtype")
        job = nat.Job()
        job.a, job.da, job.Na = a.data_ptr(), da, Na
        job.b, job.db, job.Nb = b.data_ptr(), db, Nb
        job.c, job.wc = (out.data_ptr() if n else None), out.shape[1] if n else wc
        return self.submit_job(job, keep=(a, b, out)), out

    def submit_operand(self, a: torch.Tensor, Na: int, op: "Operand",
                       out: torch.Tensor | None = None) -> tuple[int, torch.Tensor]:
        """Queue a * (op's b) against the operand's resident spectra; returns (ticket,
        output tensor).  a, out and the operand are kept alive until the ticket ends."""
        job, out = op.job(a, Na, out)
        t = nat.c_u64()
        nat.check(nat.zpm_server_submit_operand(self._h, ctypes.byref(job), ctypes.byref(t)),
                  "zpm_server_submit_operand")
        self._keep[t.value] = (a, out, op)
        return t.value, out

    def poll(self, ticket: int):
        """None while queued or running, else (status, latency_s)."""
        st, lat = nat.c_i32(), ctypes.c_double()
        nat.check(nat.zpm_server_poll(self._h, ticket, ctypes.byref(st), ctypes.byref(lat)),
                  "zpm_server_poll")
        if st.value == 1:
            return None
        self._keep.pop(ticket, None)
        return st.value, lat.value

    def wait(self, ticket: int, timeout: float = -1.0):
        """(status, latency_s) once the ticket finishes; ZpmError(EBUSY) on time-out."""
        st, lat = nat.c_i32(), ctypes.c_double()
        nat.check(nat.zpm_server_wait(self._h, ticket, timeout, ctypes.byref(st), ctypes.byref(lat)),
                  "zpm_server_wait")
        self._keep.pop(ticket, None)
        return st.value, lat.value

    def completions(self, cap: int = 4096) -> list[tuple[int, int, float]]:
        """Finished (ticket, status, latency_s) in completion order, consumed."""
        t = (nat.c_u64 * cap)()
        st = (nat.c_i32 * cap)()
        lat = (ctypes.c_double * cap)()
        n = nat.c_i64()
        nat.check(nat.zpm_server_completions(self._h, t, st, lat, cap, ctypes.byref(n)),
                  "zpm_server_completions")
        res = [(t[i], st[i], lat[i]) for i in range(n.value)]
        for tk, _, _ in res:
            self._keep.pop(tk, None)
        return res

    def stats(self) -> dict:
        r = nat.ServerReport()
        nat.check(nat.zpm_server_stats(self._h, ctypes.byref(r)), "zpm_server_stats")
        return r.as_dict()

    def reset_stats(self) -> None:
        nat.check(nat.zpm_server_reset_stats(self._h), "zpm_server_reset_stats")
