"""torch-facing API of the sample sort.

Every function here only marshals arguments (tensor pointers, the current
HIP stream, a workspace tensor) to the C ABI of ``libsamplesort.so``; all
sorting work runs in its HIP kernels.

The method (arXiv 1608.08648): sample the keys (random oversampling, Alg. 2,
or regular oversampling, Alg. 1), sort the sample, take p-1 equidistant
splitters, split the keys into p buckets (ties broken by position, Section
2.2) and sort each bucket on its own.  Results are the stable order.
"""
import ctypes

import torch

from . import native as N

_KEY = {
    torch.int32: N.SS_I32,
    torch.float32: N.SS_F32,
    torch.int64: N.SS_I64,
    torch.float64: N.SS_F64,
}
for _name, _code in (("uint32", N.SS_U32), ("uint64", N.SS_U64)):
    if hasattr(torch, _name):
        _KEY[getattr(torch, _name)] = _code

_KEY_NAMES = {"u32": N.SS_U32, "i32": N.SS_I32, "f32": N.SS_F32, "u64": N.SS_U64, "i64": N.SS_I64,
              "f64": N.SS_F64}


def key_type_of(t, key_type=None):
    """C key type of a tensor; key_type ('u32', 'i32', ...) reinterprets the
    tensor's bytes (e.g. unsigned keys held in an int32 tensor)."""
    if key_type is not None:
        kt = _KEY_NAMES[key_type] if isinstance(key_type, str) else int(key_type)
        if t.element_size() != (4 if kt <= N.SS_F32 else 8):
            raise ValueError("key_type width does not match the tensor's element size")
        return kt
    try:
        return _KEY[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported key dtype {t.dtype}")


def params(p=1024, s=8, sampling="random", seed=0x5EED, stable=True, flags=0, tile=0):
    smp = {"random": N.SS_RANDOM, "regular": N.SS_REGULAR}[sampling] if isinstance(sampling, str) else int(sampling)
    return N.Params(p=p, s=s, sampling=smp, stable=1 if stable else 0, seed=seed & (2**64 - 1), flags=flags,
                    tile=tile)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _workspace(nbytes, device, ws=None):
    nbytes = max(int(nbytes), 1)
    if ws is not None:
        if ws.numel() * ws.element_size() < nbytes or ws.data_ptr() % 256:
            raise ValueError("workspace too small or not 256-byte aligned")
        return ws
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t[off:off + nbytes]


def _pref(prm):
    """prm by reference, or NULL: the library's tuned parameters (this
    device's cached tuning table is installed on first use)."""
    if prm is None:
        from . import tune
        tune.ensure_installed()
        return None
    return ctypes.byref(prm)


def tuned_params(n, key_type, val_type=N.SS_V_NONE, segmented=False):
    """The parameters the library uses when prm is None (its tuning table)."""
    out = N.Params()
    N.check(N.lib().ss_get_tuning(1 if segmented else 0, key_type, val_type, n, ctypes.byref(out)))
    return out


def workspace_size(n, key_type, val_type=N.SS_V_NONE, prm=None):
    out = ctypes.c_size_t()
    N.check(N.lib().ss_workspace_size(n, key_type, val_type, _pref(prm), ctypes.byref(out)))
    return out.value


def stage_layout(n, key_type, val_type=N.SS_V_NONE, prm=None):
    info = N.StageInfo()
    N.check(N.lib().ss_stage_layout(n, key_type, val_type, _pref(prm), ctypes.byref(info)))
    return info


def _check_dev(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("tensors must be contiguous and on the GPU")


def _check_buf(name, t, n, width, device):
    """`t` must hold at least n elements of `width` bytes on `device` (the
    kernels read or write n elements through its pointer)."""
    if t is None:
        return
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, the keys on {device}")
    if t.element_size() != width:
        raise ValueError(f"{name} has {t.element_size()}-byte elements, {width} needed")
    if t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, {n} needed")


def sort_keys(keys, prm=None, out=None, ws=None, key_type=None, stream=None):
    """Stable ascending sort of a 1-D tensor of keys (prm None: the tuned
    parameters of n's size class)."""
    _check_dev(keys)
    kt = key_type_of(keys, key_type)
    n = keys.numel()
    out = torch.empty_like(keys) if out is None else out
    _check_dev(out)
    _check_buf("out", out, n, keys.element_size(), keys.device)
    w = _workspace(workspace_size(n, kt, N.SS_V_NONE, prm), keys.device, ws)
    N.check(N.lib().sample_sort_keys(_ptr(keys), _ptr(out), n, kt, _pref(prm), _ptr(w), w.numel(),
                                     _stream(stream)))
    return out


def sort_pairs(keys, vals=None, prm=None, iota=None, keys_out=None, vals_out=None, ws=None, key_type=None,
               stream=None):
    """Stable sort of (key, payload) pairs by key.  vals: 4- or 8-byte
    payload tensor, or None with iota='int32'/'int64' to get the stable
    sorting permutation as the payload.  prm None: tuned parameters."""
    _check_dev(keys, vals)
    kt = key_type_of(keys, key_type)
    n = keys.numel()
    if vals is None:
        if iota not in ("int32", "int64"):
            raise ValueError("give vals or iota='int32'/'int64'")
        vt = N.SS_V_IOTA32 if iota == "int32" else N.SS_V_IOTA64
        vdt = torch.int32 if iota == "int32" else torch.int64
        vals_out = torch.empty(n, dtype=vdt, device=keys.device) if vals_out is None else vals_out
    else:
        if vals.element_size() not in (4, 8):
            raise ValueError("payloads must have 4- or 8-byte elements")
        vt = {4: N.SS_V_B32, 8: N.SS_V_B64}[vals.element_size()]
        _check_buf("vals", vals, n, vals.element_size(), keys.device)
        vals_out = torch.empty_like(vals) if vals_out is None else vals_out
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    _check_dev(keys_out, vals_out)
    _check_buf("keys_out", keys_out, n, keys.element_size(), keys.device)
    _check_buf("vals_out", vals_out, n, 4 if vt in (N.SS_V_B32, N.SS_V_IOTA32) else 8, keys.device)
    w = _workspace(workspace_size(n, kt, vt, prm), keys.device, ws)
    N.check(N.lib().sample_sort_pairs(_ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out), n, kt, vt,
                                      _pref(prm), _ptr(w), w.numel(), _stream(stream)))
    return keys_out, vals_out


def segmented_workspace_size(total, nseg, max_len, key_type, val_type=N.SS_V_NONE, prm=None):
    out = ctypes.c_size_t()
    N.check(N.lib().ss_segmented_workspace_size(total, nseg, max_len, key_type, val_type,
                                                _pref(prm), ctypes.byref(out)))
    return out.value


def segmented_sort(keys, offsets, vals=None, iota=None, prm=None, max_len=0, keys_out=None, vals_out=None,
                   ws=None, key_type=None, stream=None, total=None):
    """Sort every segment [offsets[g], offsets[g+1]) of `keys` on its own.
    offsets: int64 device tensor of num_segments+1 entries.  `total`
    (= offsets[-1]) and `max_len` are host values; when not given they are
    read from `offsets` (a device-to-host copy)."""
    _check_dev(keys, offsets, vals)
    if offsets.dtype != torch.int64:
        raise TypeError("offsets must be int64")
    kt = key_type_of(keys, key_type)
    if offsets.numel() < 1 or offsets.device != keys.device:
        raise ValueError("offsets must hold num_segments + 1 entries on the keys' device")
    nseg = offsets.numel() - 1
    if total is None or not max_len:
        o = offsets.cpu()
        total = int(o[-1]) if total is None else total
        max_len = int((o[1:] - o[:-1]).max()) if (nseg > 0 and not max_len) else max_len
    if total < 0 or total > keys.numel():
        raise ValueError(f"total = {total}: the keys hold {keys.numel()}")
    if vals is None and iota is not None:
        vt = N.SS_V_IOTA32 if iota == "int32" else N.SS_V_IOTA64
        vdt = torch.int32 if iota == "int32" else torch.int64
        vals_out = torch.empty(keys.numel(), dtype=vdt, device=keys.device) if vals_out is None else vals_out
    elif vals is not None:
        if vals.element_size() not in (4, 8):
            raise ValueError("payloads must have 4- or 8-byte elements")
        vt = {4: N.SS_V_B32, 8: N.SS_V_B64}[vals.element_size()]
        _check_buf("vals", vals, total, vals.element_size(), keys.device)
        vals_out = torch.empty_like(vals) if vals_out is None else vals_out
    else:
        vt = N.SS_V_NONE
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    _check_dev(keys_out, vals_out)
    _check_buf("keys_out", keys_out, total, keys.element_size(), keys.device)
    if vt != N.SS_V_NONE:
        _check_buf("vals_out", vals_out, total, 4 if vt in (N.SS_V_B32, N.SS_V_IOTA32) else 8, keys.device)
    w = _workspace(segmented_workspace_size(total, nseg, max_len, kt, vt, prm), keys.device, ws)
    N.check(N.lib().segmented_sort(_ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out), _ptr(offsets), nseg,
                                   total, max_len, kt, vt, _pref(prm),
                                   _ptr(w), w.numel(), _stream(stream)))
    return (keys_out, vals_out) if vt != N.SS_V_NONE else keys_out


def scatter_grad(grad_y, perm, grad_x=None, stream=None):
    """grad_x[r, perm[r, j]] = grad_y[r, j] for 2-D grad_y and int64 perm."""
    _check_dev(grad_y, perm)
    if perm.dtype != torch.int64 or perm.shape != grad_y.shape or grad_y.dim() != 2:
        raise ValueError("perm must be int64 with grad_y's 2-D shape")
    grad_x = torch.empty_like(grad_y) if grad_x is None else grad_x
    _check_dev(grad_x)
    if grad_x.shape != grad_y.shape or grad_x.element_size() != grad_y.element_size() \
            or grad_x.device != grad_y.device or perm.device != grad_y.device:
        raise ValueError("grad_x must match grad_y's shape, element size and device")
    N.check(N.lib().ss_scatter_grad(_ptr(grad_y), _ptr(perm), _ptr(grad_x), grad_y.shape[0], grad_y.shape[1],
                                    grad_y.element_size(), _stream(stream)))
    return grad_x


def strings_workspace_size(n, width, prm=None):
    out = ctypes.c_size_t()
    N.check(N.lib().ss_strings_workspace_size(n, width, _pref(prm), ctypes.byref(out)))
    return out.value


def sort_strings(recs, prm=None, recs_out=None, want_sorted=True, ws=None, stream=None):
    """Stable memcmp-order sort of fixed-width byte strings: recs is a uint8
    device tensor [n, width] (width a multiple of 8).  Returns (perm int64
    [n], sorted strings [n, width] or None)."""
    _check_dev(recs)
    if recs.dtype != torch.uint8 or recs.dim() != 2:
        raise ValueError("recs must be a 2-D uint8 tensor [n, width]")
    n, width = recs.shape
    perm = torch.empty(n, dtype=torch.int64, device=recs.device)
    if want_sorted and recs_out is None:
        recs_out = torch.empty_like(recs)
    if recs_out is not None:
        _check_dev(recs_out)
        if recs_out.shape != recs.shape or recs_out.dtype != torch.uint8 or recs_out.device != recs.device:
            raise ValueError("recs_out must match recs")
    w = _workspace(strings_workspace_size(n, width, prm), recs.device, ws)
    N.check(N.lib().sample_sort_strings(_ptr(recs), _ptr(recs_out), _ptr(perm), n, width, _pref(prm), _ptr(w),
                                        w.numel(), _stream(stream)))
    return perm, recs_out


def grad_status(stream=None):
    """Wait for the stream; raise if a scatter_grad call since the last check
    met a permutation index outside its row."""
    N.check(N.lib().ss_grad_status(_stream(stream)))


def status(ws, stream=None):
    """Wait for the stream and report the device status of the last call on ws."""
    N.check(N.lib().ss_status(_ptr(ws), _stream(stream)))
    return N.last_error()


def level_stats(ws, stream=None):
    """Per split level of the last call on ws: dicts of segments, buckets,
    keys (split input) and bucket_keys (sorted in place by the level's
    bucket kernel), for the levels the call reached."""
    out = []
    for lv in range(N.SS_MAX_LEVELS):
        info = N.LevelInfo()
        N.check(N.lib().ss_level_stats(_ptr(ws), lv, ctypes.byref(info), _stream(stream)))
        if info.segments == 0:
            break
        out.append({"segments": info.segments, "buckets": info.buckets, "keys": info.keys,
                    "bucket_keys": info.bucket_keys})
    return out


def stages(keys, prm, key_type=None):
    """Run sort_keys with the stage export on and return (sorted keys, dict of
    the top-level sorted sample, splitters and bucket counts, StageInfo)."""
    if prm is None:
        prm = tuned_params(keys.numel(), key_type_of(keys, key_type))
    prm = N.Params.from_buffer_copy(prm)
    prm.flags |= N.SS_F_EXPORT_STAGES
    kt = key_type_of(keys, key_type)
    n = keys.numel()
    info = stage_layout(n, kt, N.SS_V_NONE, prm)
    w = _workspace(workspace_size(n, kt, N.SS_V_NONE, prm), keys.device)
    out = sort_keys(keys, prm, ws=w, key_type=key_type)
    torch.cuda.synchronize()
    res = {}
    if not info.direct:
        u8 = w

        def grab(off, cnt):
            return u8[off:off + 8 * cnt].view(torch.int64).cpu().numpy().view("uint64").copy()

        res["sample_ord"] = grab(info.sample_ord, info.m)
        res["sample_tag"] = grab(info.sample_tag, info.m)
        res["spl_ord"] = grab(info.spl_ord, info.p_eff - 1)
        res["spl_tag"] = grab(info.spl_tag, info.p_eff - 1)
        res["counts"] = grab(info.counts, info.p_eff).astype("int64")
    return out, res, info


def _rows_offsets(rows, cols, device):
    return torch.arange(0, (rows + 1) * cols, cols, dtype=torch.int64, device=device)


class SortFn(torch.autograd.Function):
    """Row-wise stable ascending sort of a 2-D float tensor.

    forward: (values, perm) with values[r, j] = x[r, perm[r, j]] (one
    segmented sort launch sequence over all rows, payload = in-row index).
    backward: grad_x[r, perm[r, j]] = grad_values[r, j] (a permutation, so
    no atomics)."""

    @staticmethod
    def forward(ctx, x, prm=None):
        if x.dim() != 2:
            raise ValueError("SortFn sorts the rows of a 2-D tensor")
        x = x.contiguous()
        rows, cols = x.shape
        off = _rows_offsets(rows, cols, x.device)
        vals, perm = segmented_sort(x.view(-1), off, iota="int64", prm=prm, max_len=cols, total=rows * cols)
        perm = perm.view(rows, cols)
        ctx.save_for_backward(perm)
        ctx.mark_non_differentiable(perm)
        return vals.view(rows, cols), perm

    @staticmethod
    def backward(ctx, gvals, gperm):
        (perm,) = ctx.saved_tensors
        return scatter_grad(gvals.contiguous(), perm), None


def sort(x, prm=None):
    """Differentiable row-wise sort: returns (values, perm)."""
    return SortFn.apply(x, prm)
