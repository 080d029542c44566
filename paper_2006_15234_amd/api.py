"""Torch-tensor front end of the C ABI (argument marshalling only)."""
import ctypes as C

from ._ffi import (ABSORB_CARRY, ABSORB_NONE, C128, F32, BF16, F64, Bmps, EsvdInfo, EsvdOpts,
                   Peps, Tensor)

_PREC = {"f64": F64, "f32": F32, "bf16": BF16}


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.complex128:
        return C128
    raise TypeError(f"tensors must be float64 or complex128, got {t.dtype}")


def _dev(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


_ORTH = {"cholqr": 0, "eigh": 1}
_METHOD = {"implicit": 0, "explicit": 1}


def make_opts(rank, oversample=0, power_iters=0, precision="f64", seed=0, stream_id=0,
              jacobi_max_sweeps=0, orth="cholqr", method="implicit"):
    """orth: "cholqr" (CholeskyQR2 + Householder fallback) or "eigh" (Alg. 5);
    method: "implicit" (randomized SVD, IBMPS) or "explicit" (dense SVD, BMPS)."""
    return EsvdOpts(rank=int(rank), oversample=int(oversample), power_iters=int(power_iters),
                    sketch_precision=_PREC[precision], seed=int(seed), stream_id=int(stream_id),
                    jacobi_max_sweeps=int(jacobi_max_sweeps), orth=_ORTH[orth], method=_METHOD[method],
                    reserved=0)


def _tensor_desc(t, conj, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dim() < 1 or t.dim() > 8:
        raise ValueError(f"{name}: 1 to 8 legs")
    d = Tensor(data=t.data_ptr(), ndim=t.dim(), conj=1 if conj else 0)
    for q in range(t.dim()):
        d.shape[q] = t.shape[q]
        d.strides[q] = t.stride(q)
    return d


def _network(subscripts, tensors, conj):
    conj = conj or [False] * len(tensors)
    if len(conj) != len(tensors):
        raise ValueError("one conj flag per operand")
    descs = (Tensor * len(tensors))(*[_tensor_desc(t, c, f"operand {i}")
                                      for i, (t, c) in enumerate(zip(tensors, conj))])
    lhs, rhs = subscripts.split("->")
    left, right = rhs.split("|")
    dims = {}
    for legs, t in zip(lhs.split(","), tensors):
        for c, n in zip(legs, t.shape):
            dims[c] = n
    return descs, [dims.get(c, 0) for c in left], [dims.get(c, 0) for c in right]


def einsumsvd(ctx, subscripts, *tensors, conj=None, rank, oversample=0, power_iters=0, seed=0,
              stream_id=0, absorb=ABSORB_NONE, log_scale=None, jacobi_max_sweeps=0, orth="cholqr",
              method="implicit"):
    """einsumsvd of the network `subscripts` ("ab,bc->a|c": row legs left of '|', column
    legs right of it) over strided device tensors (conj[i]: operand i enters conjugated).
    Returns (U [row dims..., m'], sigma [m'], R [m', column dims...])."""
    torch = _torch()
    if not tensors:
        raise ValueError("no operands")
    dt = _dtype_code(tensors[0])
    if any(t.dtype != tensors[0].dtype for t in tensors):
        raise TypeError("operands must share one dtype")
    descs, ldims, rdims = _network(subscripts, tensors, conj)
    o = make_opts(rank, oversample, power_iters, "f64", seed, stream_id, jacobi_max_sweeps, orth, method)
    rows, cols, mp = C.c_int64(), C.c_int64(), C.c_int64()
    ctx.check(ctx.lib.hpeps_einsumsvd_query(ctx.h, subscripts.encode(), len(tensors), descs, C.byref(o),
                                            C.byref(rows), C.byref(cols), C.byref(mp)))
    dev = tensors[0].device
    U = torch.empty((*ldims, mp.value), dtype=tensors[0].dtype, device=dev)
    sig = torch.empty((mp.value,), dtype=torch.float64, device=dev)
    R = torch.empty((mp.value, *rdims), dtype=tensors[0].dtype, device=dev)
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_einsumsvd(
        ctx.h, dt, subscripts.encode(), len(tensors), descs, C.byref(o), absorb, _dev(U, "U"),
        _dev(sig, "sigma"), _dev(R, "R"), _dev(log_scale, "log_scale") if log_scale is not None else None))
    return U, sig, R


def einsumsvd_backward(ctx, subscripts, *tensors, dU, dsigma=None, dR, conj=None, rank, oversample=0,
                       power_iters=0, seed=0, stream_id=0, absorb=ABSORB_NONE, jacobi_max_sweeps=0,
                       broadening=0.0):
    """Vector-Jacobian product of einsumsvd on the same network, operands and options
    (absorb NONE or RIGHT): the cotangents dU, dsigma (None = 0), dR of its outputs give the
    conjugate-Wirtinger gradient of the real loss with respect to every operand (contiguous,
    the operands' shapes)."""
    torch = _torch()
    if not tensors:
        raise ValueError("no operands")
    dt = _dtype_code(tensors[0])
    if any(t.dtype != tensors[0].dtype for t in tensors):
        raise TypeError("operands must share one dtype")
    descs, ldims, rdims = _network(subscripts, tensors, conj)
    o = make_opts(rank, oversample, power_iters, "f64", seed, stream_id, jacobi_max_sweeps)
    rows, cols, mp = C.c_int64(), C.c_int64(), C.c_int64()
    ctx.check(ctx.lib.hpeps_einsumsvd_query(ctx.h, subscripts.encode(), len(tensors), descs, C.byref(o),
                                            C.byref(rows), C.byref(cols), C.byref(mp)))
    if tuple(dU.shape) != (*ldims, mp.value) or tuple(dR.shape) != (mp.value, *rdims) \
            or (dsigma is not None and tuple(dsigma.shape) != (mp.value,)):
        raise ValueError("cotangent shapes do not match the outputs")
    for t, nm in ((dU, "dU"), (dR, "dR")):
        if t.dtype != tensors[0].dtype or not t.is_contiguous():
            raise TypeError(f"{nm} must be contiguous with the dtype of the operands")
    if dsigma is not None and dsigma.dtype != torch.float64:
        raise TypeError("dsigma must be float64")
    grads = [torch.empty(t.shape, dtype=t.dtype, device=t.device) for t in tensors]
    gptrs = (C.c_void_p * len(grads))(*[_dev(g, "grad") for g in grads])
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_einsumsvd_backward(
        ctx.h, dt, subscripts.encode(), len(tensors), descs, C.byref(o), absorb, float(broadening),
        _dev(dU, "dU"), _dev(dsigma, "dsigma") if dsigma is not None else None, _dev(dR, "dR"), gptrs))
    return grads


def einsumsvd_batched(ctx, subscripts, *tensors, conj=None, rank, oversample=0, power_iters=0, seed=0,
                      stream_id=0, absorb=ABSORB_NONE, log_scale=None, jacobi_max_sweeps=0, orth="cholqr",
                      method="implicit"):
    """einsumsvd of `batch` instances of the network `subscripts` at once: every operand has a
    leading instance dimension (the subscripts name the per-instance legs); instance b draws its
    sketch from stream stream_id + b.  Returns (U [B, row dims..., m'], sigma [B, m'],
    R [B, m', column dims...])."""
    torch = _torch()
    if not tensors:
        raise ValueError("no operands")
    batch = tensors[0].shape[0]
    if any(t.dim() < 2 or t.shape[0] != batch for t in tensors):
        raise ValueError("every operand needs the same leading batch dimension")
    dt = _dtype_code(tensors[0])
    if any(t.dtype != tensors[0].dtype for t in tensors):
        raise TypeError("operands must share one dtype")
    one, ldims, rdims = _network(subscripts, [t[0] for t in tensors], conj)
    descs, _, _ = _network(subscripts, tensors, conj)
    o = make_opts(rank, oversample, power_iters, "f64", seed, stream_id, jacobi_max_sweeps, orth, method)
    rows, cols, mp = C.c_int64(), C.c_int64(), C.c_int64()
    ctx.check(ctx.lib.hpeps_einsumsvd_query(ctx.h, subscripts.encode(), len(tensors), one, C.byref(o),
                                            C.byref(rows), C.byref(cols), C.byref(mp)))
    dev = tensors[0].device
    U = torch.empty((batch, *ldims, mp.value), dtype=tensors[0].dtype, device=dev)
    sig = torch.empty((batch, mp.value), dtype=torch.float64, device=dev)
    R = torch.empty((batch, mp.value, *rdims), dtype=tensors[0].dtype, device=dev)
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_einsumsvd_batched(
        ctx.h, dt, batch, subscripts.encode(), len(tensors), descs, C.byref(o), absorb, _dev(U, "U"),
        _dev(sig, "sigma"), _dev(R, "R"), _dev(log_scale, "log_scale") if log_scale is not None else None))
    return U, sig, R


def einsumsvd_zipup(ctx, V, S, T, Bra=None, *, rank, oversample=0, power_iters=0, seed=0,
                    stream_id=0, precision="f64", absorb=ABSORB_CARRY, log_scale=None,
                    jacobi_max_sweeps=0, orth="cholqr"):
    """Batched zip-up einsumsvd.  V [B,a,x,x,b,h,h], S [B,b,u,u,c], T/Bra [B,u,y,h,g,d].
    Returns (U [B,a,x,x,m'], sigma [B,m'], R [B,m',y,y,c,g,g])."""
    torch = _torch()
    Bn, a, x, x2, b, h, h2 = V.shape
    _, b2, u, u2, c = S.shape
    _, u3, y, h3, g, d = T.shape
    if not (x == x2 and h == h2 and h == h3 and b == b2 and u == u2 and u == u3
            and S.shape[0] == Bn and T.shape[0] == Bn):
        raise ValueError("inconsistent zip-up shapes")
    if Bra is not None and tuple(Bra.shape) != tuple(T.shape):
        raise ValueError("bra shape must equal ket shape")
    dt = _dtype_code(V)
    rows, cols = a * x * x, y * y * c * g * g
    k = min(rank + oversample, rows, cols)
    mp = min(rank, k)
    U = torch.empty((Bn, a, x, x, mp), dtype=V.dtype, device=V.device)
    sig = torch.empty((Bn, mp), dtype=torch.float64, device=V.device)
    R = torch.empty((Bn, mp, y, y, c, g, g), dtype=V.dtype, device=V.device)
    dims = (C.c_int64 * 9)(a, x, b, h, u, c, y, g, d)
    o = make_opts(rank, oversample, power_iters, precision, seed, stream_id, jacobi_max_sweeps, orth)
    ctx.sync_stream()
    ls = _dev(log_scale, "log_scale") if log_scale is not None else None
    ctx.check(ctx.lib.hpeps_einsumsvd_zipup(
        ctx.h, Bn, dt, dims, _dev(V, "V"), _dev(S, "S"), _dev(T, "T"),
        _dev(Bra, "Bra") if Bra is not None else None, C.byref(o), absorb,
        _dev(U, "U"), _dev(sig, "sigma"), _dev(R, "R"), ls))
    return U, sig, R


def einsumsvd_pair(ctx, Bl, Br, T1, T2, *, rank, oversample=0, power_iters=0, seed=0,
                   stream_id=0, precision="f64", absorb=ABSORB_CARRY, jacobi_max_sweeps=0,
                   orth="cholqr"):
    """Batched pair einsumsvd.  Bl, Br [B,m,D,D,m]; T1 [B,D,D,1,D,d]; T2 [B,D,D,D,1,d].
    Returns (U [B,m,D,D,m'], sigma [B,m'], R [B,m',D,D,m])."""
    torch = _torch()
    Bn, m, D, _, _ = Bl.shape
    d = T1.shape[-1]
    if tuple(Br.shape) != tuple(Bl.shape) or tuple(T1.shape) != (Bn, D, D, 1, D, d) \
            or tuple(T2.shape) != (Bn, D, D, D, 1, d):
        raise ValueError("inconsistent pair shapes")
    dt = _dtype_code(Bl)
    rows = cols = m * D * D
    k = min(rank + oversample, rows, cols)
    mp = min(rank, k)
    U = torch.empty((Bn, m, D, D, mp), dtype=Bl.dtype, device=Bl.device)
    sig = torch.empty((Bn, mp), dtype=torch.float64, device=Bl.device)
    R = torch.empty((Bn, mp, D, D, m), dtype=Bl.dtype, device=Bl.device)
    dims = (C.c_int64 * 3)(m, D, d)
    o = make_opts(rank, oversample, power_iters, precision, seed, stream_id, jacobi_max_sweeps, orth)
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_einsumsvd_pair(
        ctx.h, Bn, dt, dims, _dev(Bl, "Bl"), _dev(Br, "Br"), _dev(T1, "T1"), _dev(T2, "T2"),
        C.byref(o), absorb, _dev(U, "U"), _dev(sig, "sigma"), _dev(R, "R")))
    return U, sig, R


def einsumsvd_pair_backward(ctx, Bl, Br, T1, T2, dU, dsigma, dR, *, rank, oversample=0,
                            power_iters=0, seed=0, stream_id=0, absorb=ABSORB_NONE,
                            jacobi_max_sweeps=0, broadening=0.0):
    """Vector-Jacobian product of einsumsvd_pair (FP64 sketch, absorb NONE or RIGHT): the
    cotangents dU, dsigma (None = 0), dR of its outputs give (gBl, gBr, gT1, gT2), the
    conjugate-Wirtinger gradients of the real loss with respect to the four inputs.
    broadening: Lorentzian width of the SVD backward's 1/(s_j^2 - s_i^2), relative to
    s_1^4 (0 = exact derivative)."""
    torch = _torch()
    Bn, m, D, _, _ = Bl.shape
    d = T1.shape[-1]
    rows = m * D * D
    k = min(rank + oversample, rows, rows)
    mp = min(rank, k)
    if tuple(dU.shape) != (Bn, m, D, D, mp) or tuple(dR.shape) != (Bn, mp, D, D, m) \
            or (dsigma is not None and tuple(dsigma.shape) != (Bn, mp)):
        raise ValueError("cotangent shapes do not match the outputs")
    dt = _dtype_code(Bl)
    for t, nm in ((dU, "dU"), (dR, "dR")):
        if t.dtype != Bl.dtype:
            raise TypeError(f"{nm} must have the dtype of the inputs")
    if dsigma is not None and dsigma.dtype != torch.float64:
        raise TypeError("dsigma must be float64")
    grads = [torch.empty_like(t) for t in (Bl, Br, T1, T2)]
    dims = (C.c_int64 * 3)(m, D, d)
    o = make_opts(rank, oversample, power_iters, "f64", seed, stream_id, jacobi_max_sweeps)
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_einsumsvd_pair_backward(
        ctx.h, Bn, dt, dims, _dev(Bl, "Bl"), _dev(Br, "Br"), _dev(T1, "T1"), _dev(T2, "T2"),
        C.byref(o), absorb, float(broadening), _dev(dU, "dU"), _dev(dsigma, "dsigma") if dsigma is not None else None,
        _dev(dR, "dR"), *[_dev(g, "grad") for g in grads]))
    return tuple(grads)


def einsumsvd_pair_autograd(ctx, Bl, Br, T1, T2, *, rank, oversample=0, power_iters=0, seed=0,
                            stream_id=0, absorb=ABSORB_NONE, jacobi_max_sweeps=0, broadening=0.0):
    """einsumsvd_pair as a differentiable torch function: forward and backward both run
    in the library (the backward recomputes the forward with the same sketch)."""
    torch = _torch()
    kw = dict(rank=rank, oversample=oversample, power_iters=power_iters, seed=seed,
              stream_id=stream_id, absorb=absorb, jacobi_max_sweeps=jacobi_max_sweeps)

    class _PairEsvd(torch.autograd.Function):
        @staticmethod
        def forward(fctx, Bl, Br, T1, T2):
            fctx.save_for_backward(Bl, Br, T1, T2)
            return einsumsvd_pair(ctx, Bl, Br, T1, T2, precision="f64", **kw)

        @staticmethod
        def backward(fctx, gU, gs, gR):
            Bl, Br, T1, T2 = fctx.saved_tensors
            mp = min(rank, min(rank + oversample, Bl.shape[1] * Bl.shape[2] ** 2))
            shapeU = (Bl.shape[0], Bl.shape[1], Bl.shape[2], Bl.shape[2], mp)
            shapeR = (Bl.shape[0], mp, Bl.shape[2], Bl.shape[2], Bl.shape[1])
            gU = torch.zeros(shapeU, dtype=Bl.dtype, device=Bl.device) if gU is None \
                else gU.contiguous()
            gR = torch.zeros(shapeR, dtype=Bl.dtype, device=Bl.device) if gR is None \
                else gR.contiguous()
            gs = None if gs is None else gs.contiguous()
            return einsumsvd_pair_backward(ctx, Bl.contiguous(), Br.contiguous(), T1.contiguous(),
                                           T2.contiguous(), gU, gs, gR, broadening=broadening,
                                           **kw)

    return _PairEsvd.apply(Bl, Br, T1, T2)


def einsumsvd_autograd(ctx, subscripts, *tensors, conj=None, rank, oversample=0, power_iters=0, seed=0,
                       stream_id=0, absorb=ABSORB_NONE, jacobi_max_sweeps=0, broadening=0.0):
    """einsumsvd of the network `subscripts` as a differentiable torch function (absorb NONE
    or RIGHT): forward and backward both run in the library (the backward recomputes the
    forward with the same sketch), and gradients flow to every operand."""
    torch = _torch()
    kw = dict(rank=rank, oversample=oversample, power_iters=power_iters, seed=seed,
              stream_id=stream_id, absorb=absorb, jacobi_max_sweeps=jacobi_max_sweeps)

    class _NetworkEsvd(torch.autograd.Function):
        @staticmethod
        def forward(fctx, *ts):
            fctx.save_for_backward(*ts)
            U, s, R = einsumsvd(ctx, subscripts, *ts, conj=conj, **kw)
            fctx.shapes = (tuple(U.shape), tuple(R.shape))
            return U, s, R

        @staticmethod
        def backward(fctx, gU, gs, gR):
            ts = fctx.saved_tensors
            su, sr = fctx.shapes
            dt, dev = ts[0].dtype, ts[0].device
            gU = torch.zeros(su, dtype=dt, device=dev) if gU is None else gU.contiguous()
            gR = torch.zeros(sr, dtype=dt, device=dev) if gR is None else gR.contiguous()
            gs = None if gs is None else gs.contiguous()
            return tuple(einsumsvd_backward(ctx, subscripts, *ts, dU=gU, dsigma=gs, dR=gR, conj=conj,
                                            broadening=broadening, **kw))

    return _NetworkEsvd.apply(*tensors)


def sketch(ctx, n, k, batch=1, seed=0, stream_id=0, precision="f64", device="cuda"):
    """The sketch an einsumsvd with (seed, stream_id) draws: [batch, n, k]."""
    torch = _torch()
    dt = torch.float64 if precision == "f64" else torch.float32
    out = torch.empty((batch, n, k), dtype=dt, device=device)
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_sketch(ctx.h, _PREC[precision], n, k, batch, seed, stream_id,
                                   _dev(out, "out")))
    return out


class ProfileEntry(C.Structure):
    _fields_ = [("name", C.c_char * 64), ("launches", C.c_int64), ("ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


def profile_start(ctx, filter=None):
    """Start live per-kernel timing with HIP events (see hpeps_profile_start)."""
    ctx.check(ctx.lib.hpeps_profile_start(ctx.h, filter.encode() if filter else None))


def profile_stop(ctx):
    ctx.check(ctx.lib.hpeps_profile_stop(ctx.h))


def profile_by_shape(ctx, on=True):
    """GEMM class names with the product's M, N, K and batch (see hpeps_profile_by_shape)."""
    ctx.check(ctx.lib.hpeps_profile_by_shape(ctx.h, 1 if on else 0))


def profile_read(ctx):
    """Synchronises and returns {class: dict(launches, ms, flops, bytes)}; clears."""
    buf = (ProfileEntry * 128)()
    n = C.c_int32()
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_profile_read(ctx.h, 128, C.cast(buf, C.c_void_p), C.byref(n)))
    return {buf[i].name.decode(): dict(launches=buf[i].launches, ms=buf[i].ms, flops=buf[i].flops,
                                       bytes=buf[i].bytes) for i in range(min(n.value, 128))}


def autotune_enable(ctx, on=True):
    """Turns the per-shape GEMM autotuner of the context on or off."""
    ctx.check(ctx.lib.hpeps_autotune_enable(ctx.h, 1 if on else 0))


def autotune_export(ctx):
    """The tuned GEMM variants as JSON text."""
    need = C.c_int64()
    ctx.check(ctx.lib.hpeps_autotune_export(ctx.h, None, 0, C.byref(need)))
    buf = C.create_string_buffer(need.value)
    ctx.check(ctx.lib.hpeps_autotune_export(ctx.h, buf, need.value, C.byref(need)))
    return buf.value.decode()


def autotune_import(ctx, text):
    """Merges tuned variants from JSON text written by ``autotune_export``."""
    ctx.check(ctx.lib.hpeps_autotune_import(ctx.h, text.encode()))


def autotune_save(ctx, path):
    with open(path, "w") as f:
        f.write(autotune_export(ctx))


def autotune_load(ctx, path):
    with open(path) as f:
        autotune_import(ctx, f.read())


def workspace_peak(ctx, reset=False):
    """High-water mark of the library's workspace (bytes) on this context."""
    b = C.c_int64()
    ctx.check(ctx.lib.hpeps_workspace_peak(ctx.h, C.byref(b), 1 if reset else 0))
    return b.value


def get_info(ctx):
    info = EsvdInfo()
    ctx.check(ctx.lib.hpeps_get_info(ctx.h, C.byref(info)))
    return {f: getattr(info, f) for f, _ in EsvdInfo._fields_}


# ---------------------------------------------------------------------------
# lattice-level calls

def _peps_struct(sites, dtype_code, keep):
    """sites: list of rows of device tensors [u,d,l,r,p]."""
    nrow, ncol = len(sites), len(sites[0])
    ptrs = (C.c_void_p * (nrow * ncol))()
    shapes = (C.c_int64 * (nrow * ncol * 5))()
    for i in range(nrow):
        for j in range(ncol):
            t = sites[i][j]
            ptrs[i * ncol + j] = _dev(t, f"site ({i},{j})").value
            for q in range(5):
                shapes[(i * ncol + j) * 5 + q] = t.shape[q]
    keep.extend([ptrs, shapes])
    return Peps(nrow=nrow, ncol=ncol, dtype=dtype_code, reserved=0,
                sites=C.cast(ptrs, C.POINTER(C.c_void_p)), shapes=C.cast(shapes, C.POINTER(C.c_int64)))


def peps_norm(ctx, ket, bra=None, *, rank, oversample=0, power_iters=0, seed=0, precision="f64",
              jacobi_max_sweeps=0, orth="cholqr"):
    """<bra|ket> by boundary MPS.  Returns (log|v|, phase as complex)."""
    keep = []
    dt = _dtype_code(ket[0][0])
    pk = _peps_struct(ket, dt, keep)
    pb = _peps_struct(bra, dt, keep) if bra is not None else None
    o = make_opts(rank, oversample, power_iters, precision, seed, 0, jacobi_max_sweeps, orth)
    ln = C.c_double()
    ph = (C.c_double * 2)()
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_peps_norm(ctx.h, C.byref(pk), C.byref(pb) if pb is not None else None,
                                      C.byref(o), C.byref(ln), ph))
    return ln.value, complex(ph[0], ph[1])


def peps_amplitude(ctx, ket, bits, *, rank, oversample=0, power_iters=0, seed=0, jacobi_max_sweeps=0,
                   method="implicit"):
    """<bits|psi> by the one-layer boundary MPS (bits: one int per site, row-major).
    Returns (log|a|, phase as complex); (-inf, 0) for an exactly zero slice."""
    keep = []
    dt = _dtype_code(ket[0][0])
    pk = _peps_struct(ket, dt, keep)
    nsites = len(ket) * len(ket[0])
    if len(bits) != nsites:
        raise ValueError("bits needs one entry per site")
    b = (C.c_int32 * nsites)(*[int(v) for v in bits])
    o = make_opts(rank, oversample, power_iters, "f64", seed, 0, jacobi_max_sweeps, method=method)
    la = C.c_double()
    ph = (C.c_double * 2)()
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_peps_amplitude(ctx.h, C.byref(pk), b, C.byref(o), C.byref(la), ph))
    return la.value, complex(ph[0], ph[1])


def peps_amplitudes(ctx, ket, states, *, rank, oversample=0, power_iters=0, seed=0, jacobi_max_sweeps=0,
                    method="implicit"):
    """<bits|psi> for a batch of basis states (``states``: sequences of one int per
    site, row-major), computed in lockstep.  Returns (log|a| list, phase list)."""
    keep = []
    dt = _dtype_code(ket[0][0])
    pk = _peps_struct(ket, dt, keep)
    nsites = len(ket) * len(ket[0])
    flat = [int(v) for b in states for v in b]
    n = len(states)
    if n < 1 or len(flat) != n * nsites:
        raise ValueError("states needs one entry per site for every state")
    b = (C.c_int32 * len(flat))(*flat)
    o = make_opts(rank, oversample, power_iters, "f64", seed, 0, jacobi_max_sweeps, method=method)
    la = (C.c_double * n)()
    ph = (C.c_double * (2 * n))()
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_peps_amplitudes(ctx.h, C.byref(pk), n, b, C.byref(o), la, ph))
    return list(la), [complex(ph[2 * t], ph[2 * t + 1]) for t in range(n)]


def boundary_contract_row(ctx, bnd, ket, bra=None, *, row, direction, rank, oversample=0,
                          power_iters=0, seed=0, stream_id=0, precision="f64", out_capacity=None):
    """Absorbs row ``row`` of the lattice ``ket`` (list of rows of device site
    tensors; ``bra`` likewise, None for conj(ket)) into a boundary MPS (list of
    [mL,x,X,mR] device tensors).  Returns (new boundary list, log scale added)."""
    torch = _torch()
    keep = []
    ket_row = ket[row]
    dt = _dtype_code(ket_row[0])
    ncol = len(ket_row)
    bp = (C.c_void_p * ncol)(*[_dev(t, "bnd").value for t in bnd])
    bs = (C.c_int64 * (4 * ncol))(*[s for t in bnd for s in t.shape])
    bin_ = Bmps(ncol=ncol, dtype=dt, tensors=C.cast(bp, C.POINTER(C.c_void_p)),
                shapes=C.cast(bs, C.POINTER(C.c_int64)), capacity=None)
    pk = _peps_struct(ket, dt, keep)
    pb = _peps_struct(bra, dt, keep) if bra is not None else None
    # output capacity: m' <= rank + 0 per bond; down legs of the row
    outs = []
    for j, T in enumerate(ket_row):
        mL = 1 if j == 0 else rank
        mR = 1 if j == ncol - 1 else rank
        cap = mL * T.shape[1] * T.shape[1] * mR if out_capacity is None else out_capacity[j]
        outs.append(torch.empty(cap, dtype=ket_row[0].dtype, device=ket_row[0].device))
    op = (C.c_void_p * ncol)(*[t.data_ptr() for t in outs])
    oshape = (C.c_int64 * (4 * ncol))()
    ocap = (C.c_int64 * ncol)(*[t.numel() for t in outs])
    bout = Bmps(ncol=ncol, dtype=dt, tensors=C.cast(op, C.POINTER(C.c_void_p)),
                shapes=C.cast(oshape, C.POINTER(C.c_int64)), capacity=C.cast(ocap, C.POINTER(C.c_int64)))
    o = make_opts(rank, oversample, power_iters, precision, seed, stream_id)
    ls = C.c_double(0.0)
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_boundary_contract_row(ctx.h, C.byref(bin_), C.byref(pk),
                                                  C.byref(pb) if pb is not None else None, row,
                                                  direction, C.byref(o), C.byref(bout), C.byref(ls)))
    res = []
    for j in range(ncol):
        shp = tuple(oshape[4 * j:4 * j + 4])
        n = shp[0] * shp[1] * shp[2] * shp[3]
        res.append(outs[j][:n].view(shp))
    return res, ls.value


def _terms_arrays(terms):
    import numpy as np
    n = len(terms)
    ns = (C.c_int32 * n)()
    st = (C.c_int32 * (4 * n))()
    offs = (C.c_int64 * n)()
    flat = []
    off = 0
    for t, (sites, op) in enumerate(terms):
        ns[t] = len(sites)
        for q, (i, j) in enumerate(sites):
            st[4 * t + 2 * q] = i
            st[4 * t + 2 * q + 1] = j
        a = np.asarray(op, dtype=np.complex128).ravel()
        offs[t] = off
        flat.append(np.stack([a.real, a.imag], axis=-1).ravel())
        off += a.size
    ops = np.ascontiguousarray(np.concatenate(flat)) if flat else np.zeros(2)
    return n, ns, st, offs, ops


def peps_energy(ctx, ket, terms, *, rank, oversample=0, power_iters=0, seed=0, precision="f64"):
    """terms: list of (sites, op) with op a [2,2] or [2,2,2,2] complex array (host).
    Returns (energy complex, per-term complex list)."""
    keep = []
    dt = _dtype_code(ket[0][0])
    pk = _peps_struct(ket, dt, keep)
    n, ns, st, offs, ops = _terms_arrays(terms)
    o = make_opts(rank, oversample, power_iters, precision, seed, 0)
    e = (C.c_double * 2)()
    per = (C.c_double * (2 * n))()
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_peps_energy(ctx.h, C.byref(pk), n, ns, st,
                                        ops.ctypes.data_as(C.POINTER(C.c_double)), offs,
                                        C.byref(o), e, per))
    return complex(e[0], e[1]), [complex(per[2 * t], per[2 * t + 1]) for t in range(n)]


def peps_energy_uncached(ctx, ket, terms, *, rank, oversample=0, power_iters=0, seed=0):
    """Eq. 5 without cached environments: every term <psi|H_t psi> / <psi|psi> is its
    own boundary contraction of the exactly applied H_t psi.  Same terms and
    returns as peps_energy."""
    keep = []
    dt = _dtype_code(ket[0][0])
    pk = _peps_struct(ket, dt, keep)
    n, ns, st, offs, ops = _terms_arrays(terms)
    o = make_opts(rank, oversample, power_iters, "f64", seed, 0)
    e = (C.c_double * 2)()
    per = (C.c_double * (2 * max(n, 1)))()
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_peps_energy_uncached(ctx.h, C.byref(pk), n, ns, st,
                                                 ops.ctypes.data_as(C.POINTER(C.c_double)), offs,
                                                 C.byref(o), e, per))
    return complex(e[0], e[1]), [complex(per[2 * t], per[2 * t + 1]) for t in range(n)]


def peps_trotter_expectation(ctx, ket, gates, tau, *, rank, oversample=0, power_iters=0, seed=0):
    """Eq. 6: (<psi| prod_j G_j |psi> / <psi|psi> - 1) / tau with gates
    [((i1, j1), (i2, j2)), G] (G = e^{tau H_j} as [d,d,d,d], applied exactly in
    the order given).  Returns (estimate, overlap ratio), both complex."""
    keep = []
    dt = _dtype_code(ket[0][0])
    pk = _peps_struct(ket, dt, keep)
    n, _, st, _, ops = _terms_arrays(gates)
    o = make_opts(rank, oversample, power_iters, "f64", seed, 0)
    est = (C.c_double * 2)()
    rat = (C.c_double * 2)()
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_peps_trotter_expectation(ctx.h, C.byref(pk), n, st,
                                                     ops.ctypes.data_as(C.POINTER(C.c_double)), float(tau),
                                                     C.byref(o), est, rat))
    return complex(est[0], est[1]), complex(rat[0], rat[1])


def _grad_buffers(ket):
    torch = _torch()
    grads = [[torch.empty_like(t) for t in row] for row in ket]
    flat = [g for row in grads for g in row]
    arr = (C.c_void_p * len(flat))(*[_dev(g, "grad").value for g in flat])
    return grads, arr


def peps_energy_backward(ctx, ket, terms, *, rank, oversample=0, power_iters=0, seed=0,
                         broadening=0.0):
    """Gradient of Re E, E = <psi|H|psi> / <psi|psi> from the cached-environment
    contraction (same terms and options as peps_energy, FP64 sketch), with respect to
    every site tensor (conjugate Wirtinger for complex sites).  Returns (energy complex,
    gradients as rows of device tensors shaped like the sites)."""
    keep = []
    dt = _dtype_code(ket[0][0])
    pk = _peps_struct(ket, dt, keep)
    n, ns, st, offs, ops = _terms_arrays(terms)
    o = make_opts(rank, oversample, power_iters, "f64", seed, 0)
    grads, arr = _grad_buffers(ket)
    e = (C.c_double * 2)()
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_peps_energy_backward(
        ctx.h, C.byref(pk), n, ns, st, ops.ctypes.data_as(C.POINTER(C.c_double)), offs, C.byref(o),
        float(broadening), C.cast(arr, C.POINTER(C.c_void_p)), e))
    return complex(e[0], e[1]), grads


def peps_energy_autograd(ctx, ket, terms, *, rank, oversample=0, power_iters=0, seed=0,
                         broadening=0.0):
    """Re E as a differentiable torch scalar of the site tensors (rows of device tensors
    with requires_grad): the forward call runs the library's energy with its reverse-mode
    gradient in one pass (the gradient needs the forward anyway), the backward scales that
    gradient by the incoming cotangent."""
    torch = _torch()
    nrow, ncol = len(ket), len(ket[0])
    kw = dict(rank=rank, oversample=oversample, power_iters=power_iters, seed=seed,
              broadening=broadening)

    class _Energy(torch.autograd.Function):
        @staticmethod
        def forward(fctx, *sites):
            lat = [[sites[i * ncol + j].detach().contiguous() for j in range(ncol)]
                   for i in range(nrow)]
            e, grads = peps_energy_backward(ctx, lat, terms, **kw)
            fctx.save_for_backward(*[g for row in grads for g in row])
            return torch.tensor(e.real, dtype=torch.float64, device=sites[0].device)

        @staticmethod
        def backward(fctx, g):
            return tuple(g * t for t in fctx.saved_tensors)

    return _Energy.apply(*[t for row in ket for t in row])


def peps_norm_backward(ctx, ket, *, rank, oversample=0, power_iters=0, seed=0, broadening=0.0):
    """Gradient of log <psi|psi> (boundary-MPS contraction, FP64 sketch) with respect to
    every site tensor.  Returns (log <psi|psi>, gradients as rows of device tensors)."""
    keep = []
    dt = _dtype_code(ket[0][0])
    pk = _peps_struct(ket, dt, keep)
    o = make_opts(rank, oversample, power_iters, "f64", seed, 0)
    grads, arr = _grad_buffers(ket)
    ln = C.c_double()
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_peps_norm_backward(ctx.h, C.byref(pk), C.byref(o), float(broadening),
                                               C.cast(arr, C.POINTER(C.c_void_p)), C.byref(ln)))
    return ln.value, grads


def apply_one_site_gate(ctx, sites, i, j, G):
    """Eq. 3 on sites[i][j] (list of rows of device tensors [u,d,l,r,p]) with
    the device d x d gate G (out, in); returns the updated site tensor (a new
    device tensor; the others are unchanged)."""
    torch = _torch()
    T = sites[i][j].contiguous()
    out = torch.empty_like(T)
    Gd = G.contiguous().to(T.dtype)
    dims = (C.c_int64 * 5)(*T.shape)
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_apply_one_site_gate(ctx.h, _dtype_code(T), dims, _dev(T, "site"), _dev(Gd, "G"),
                                                _dev(out, "out")))
    return out


def apply_two_site_gate(ctx, sites, i, j, axis, G, max_rank, noalloc=False):
    """QR-SVD update (Alg. 1) of sites[i][j] and its right (axis 0) or lower
    (axis 1) neighbour with the gate G[out1,out2,in1,in2] (device tensor).
    ``sites`` is a list of rows of device tensors [u,d,l,r,p]; returns
    (new lattice as a list of rows, kept singular values on the device).
    noalloc selects hpeps_apply_two_site_gate_noalloc (the library's buffers
    from its static device scratch instead of its workspace)."""
    torch = _torch()
    nrow, ncol = len(sites), len(sites[0])
    d = sites[0][0].shape[4]
    cap = max_rank ** 4 * d
    bufs = [[torch.zeros(cap, dtype=sites[0][0].dtype, device=sites[0][0].device) for _ in range(ncol)]
            for _ in range(nrow)]
    for r in range(nrow):
        for c in range(ncol):
            bufs[r][c][:sites[r][c].numel()] = sites[r][c].reshape(-1)
    ptrs = (C.c_void_p * (nrow * ncol))(*[bufs[r][c].data_ptr() for r in range(nrow) for c in range(ncol)])
    shapes = (C.c_int64 * (nrow * ncol * 5))(*[s for r in range(nrow) for c in range(ncol)
                                               for s in sites[r][c].shape])
    capa = (C.c_int64 * (nrow * ncol))(*([cap] * (nrow * ncol)))
    pk = Peps(nrow=nrow, ncol=ncol, dtype=_dtype_code(sites[0][0]), reserved=0,
              sites=C.cast(ptrs, C.POINTER(C.c_void_p)), shapes=C.cast(shapes, C.POINTER(C.c_int64)))
    sig = torch.zeros(max_rank, dtype=torch.float64, device=sites[0][0].device)
    nb = C.c_int64()
    Gd = G.contiguous()
    ctx.sync_stream()
    fn = ctx.lib.hpeps_apply_two_site_gate_noalloc if noalloc else ctx.lib.hpeps_apply_two_site_gate
    ctx.check(fn(ctx.h, C.byref(pk), capa, i, j, axis, _dev(Gd, "G"), max_rank, C.byref(nb),
                 _dev(sig, "sigma")))
    out = []
    for r in range(nrow):
        row = []
        for c in range(ncol):
            shp = tuple(shapes[(r * ncol + c) * 5:(r * ncol + c) * 5 + 5])
            n = shp[0] * shp[1] * shp[2] * shp[3] * shp[4]
            row.append(bufs[r][c][:n].view(shp))
        out.append(row)
    return out, sig[:nb.value]


class ItePlan:
    """Batched imaginary-time-evolution sweeps (TEBD with QR-SVD updates).

    peps: list of rows of device tensors (initial state, bonds <= max_rank);
    gates: device tensor [n_gates, d, d, d, d]; bond_gate: gate index of every
    bond in layer order (horizontal even columns, horizontal odd columns,
    vertical even rows, vertical odd rows)."""

    def __init__(self, ctx, peps, gates, bond_gate, max_rank):
        keep = []
        self._setup(ctx, peps, max_rank)
        pk = _peps_struct(peps, _dtype_code(peps[0][0]), keep)
        bg = (C.c_int32 * len(bond_gate))(*bond_gate)
        self.gates = gates.contiguous()
        h = C.c_void_p()
        ctx.sync_stream()
        ctx.check(ctx.lib.hpeps_ite_plan_create(ctx.h, C.byref(pk), self.gates.shape[0],
                                                _dev(self.gates, "gates"), bg, max_rank, C.byref(h)))
        self.h = h
        self._count()

    def _setup(self, ctx, peps, max_rank):
        self.ctx = ctx
        self.nrow, self.ncol = len(peps), len(peps[0])
        self.dtype = peps[0][0].dtype
        self.device = peps[0][0].device
        self.max_rank = int(max_rank)

    def _count(self):
        nl, nb = C.c_int32(), C.c_int32()
        self.ctx.check(self.ctx.lib.hpeps_ite_plan_layers(self.h, C.byref(nl), C.byref(nb)))
        self.n_layers, self.n_bonds = nl.value, nb.value

    def run(self, n_sweeps, use_graph=True, per_bond=False):
        """use_graph: replay the captured sweep graph; per_bond: the plain form,
        one launch per bond (no graph)."""
        self.ctx.sync_stream()
        mode = 2 if per_bond else (1 if use_graph else 0)
        self.ctx.check(self.ctx.lib.hpeps_ite_run(self.h, n_sweeps, mode))

    def spectra(self):
        """Kept singular values of every bond update of the last sweep, layer
        order: device tensor [n_bonds, max_rank] (zero-padded)."""
        torch = _torch()
        out = torch.zeros((self.n_bonds, self.max_rank), dtype=torch.float64, device=self.device)
        self.ctx.sync_stream()
        self.ctx.check(self.ctx.lib.hpeps_ite_spectra(self.h, _dev(out, "spectra")))
        return out

    def shapes(self):
        n = self.nrow * self.ncol
        shp = (C.c_int64 * (5 * n))()
        self.ctx.check(self.ctx.lib.hpeps_ite_get_state(self.h, shp, None))
        return [tuple(shp[5 * q:5 * q + 5]) for q in range(n)]

    def state(self):
        """Copies of the current site tensors (list of rows of device tensors)."""
        torch = _torch()
        shp = self.shapes()
        outs = [torch.empty(s, dtype=self.dtype, device=self.device) for s in shp]
        ptrs = (C.c_void_p * len(outs))(*[t.data_ptr() for t in outs])
        shp2 = (C.c_int64 * (5 * len(outs)))()
        self.ctx.check(self.ctx.lib.hpeps_ite_get_state(self.h, shp2, ptrs))
        return [outs[r * self.ncol:(r + 1) * self.ncol] for r in range(self.nrow)]

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.ctx.lib.hpeps_ite_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CircuitPlan(ItePlan):
    """A sweep over an arbitrary gate list (hpeps_circuit_plan_create): ops is a
    list of (2, (i1, j1), (i2, j2), gate) two-site operations (any two sites:
    non-neighbours run as SWAP chains) and (1, (i, j), gate) one-site
    operations, in order; gates2 [n2, d, d, d, d] and gates1 [n1, d, d] are
    host float64 arrays.  run / spectra / state / close as for ItePlan."""

    def __init__(self, ctx, peps, ops, gates2, gates1, max_rank):
        import numpy as np
        keep = []
        self._setup(ctx, peps, max_rank)
        pk = _peps_struct(peps, _dtype_code(peps[0][0]), keep)
        flat = []
        for op in ops:
            if op[0] == 1:
                flat += [1, op[1][0], op[1][1], 0, 0, op[2]]
            else:
                flat += [2, op[1][0], op[1][1], op[2][0], op[2][1], op[3]]
        arr = (C.c_int32 * len(flat))(*flat)
        g2 = np.ascontiguousarray(np.asarray(gates2, dtype=np.float64).reshape(-1))
        g1 = np.ascontiguousarray(np.asarray(gates1, dtype=np.float64).reshape(-1))
        d = peps[0][0].shape[4]
        h = C.c_void_p()
        ctx.sync_stream()
        ctx.check(ctx.lib.hpeps_circuit_plan_create(
            ctx.h, C.byref(pk), g2.size // d ** 4, g2.ctypes.data_as(C.POINTER(C.c_double)),
            g1.size // d ** 2, g1.ctypes.data_as(C.POINTER(C.c_double)), len(ops), arr, max_rank, C.byref(h)))
        self.h = h
        self._count()
