"""Python binding of libhers (argument marshalling only).

Every step of keygen, encryption, search and decryption runs in the HIP
kernels of libhers.so; this module allocates device memory through PyTorch,
passes raw pointers and the current HIP stream, and checks return codes.  It
raises if the library is missing: there is no CPU fallback.

The call names follow include/hers.h: keygen, load_keys, encrypt_gallery,
encrypt_probe, search, search_batch, decrypt_scores.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhers.so")

c_u32, c_u64, c_i32, c_i64, c_vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
MAX_QPRIMES = 8


class HersParams(ctypes.Structure):
    _fields_ = [("n", c_u32), ("k", c_u32), ("qbits", c_u32 * MAX_QPRIMES), ("t_bits", c_u32),
                ("w_bits", c_u32), ("d_max", c_u32), ("feature_bound", c_u32)]


class HersInfo(ctypes.Structure):
    _fields_ = [("n", c_u32), ("k", c_u32), ("q", c_u64 * MAX_QPRIMES), ("t", c_u64), ("num_digits", c_u32),
                ("num_aux", c_u32), ("aux", c_u64 * 32), ("log2_q", ctypes.c_double), ("log2_aux", ctypes.c_double),
                ("d_max", c_u32), ("feature_bound", c_u32)]


EXPORTS = {
    "hers_last_error": (ctypes.c_char_p, []),
    "hers_params_resolve": (c_i32, [ctypes.POINTER(HersParams), ctypes.POINTER(HersInfo)]),
    "hers_ctx_create": (c_i32, [ctypes.POINTER(HersParams), c_i32, ctypes.POINTER(c_vp)]),
    "hers_ctx_destroy": (None, [c_vp]),
    "hers_ctx_info": (c_i32, [c_vp, ctypes.POINTER(HersInfo)]),
    "hers_blocks": (c_u64, [c_vp, c_i64]),
    "hers_ct_words": (c_u64, [c_vp]),
    "hers_pk_words": (c_u64, [c_vp]),
    "hers_rlk_words": (c_u64, [c_vp]),
    "hers_gallery_words": (c_u64, [c_vp, c_i64, c_i32]),
    "hers_probe_words": (c_u64, [c_vp, c_i32]),
    "hers_workspace_bytes": (c_u64, [c_vp, ctypes.c_int, c_i64, c_i32]),
    "hers_keygen": (c_i32, [c_vp, c_u64, c_vp, c_vp, c_vp, c_vp]),
    "hers_load_keys": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "hers_enroll_append": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_i64, c_i32, c_u64, c_vp, c_vp, c_vp,
                                    ctypes.c_size_t, c_vp]),
    "hers_search_literal": (c_i32, [c_vp, c_vp, c_u64, c_i64, c_i32, c_vp, c_u64, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "hers_rotation_key_words": (c_u64, [c_vp, c_i32]),
    "hers_rotation_keygen": (c_i32, [c_vp, c_u64, c_i32, c_vp, c_vp]),
    "hers_rerank_encrypt": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_i32, c_i32, ctypes.c_int, c_u64, c_vp, c_vp, c_vp,
                                     ctypes.c_size_t, c_vp]),
    "hers_rerank": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_i32, c_vp, c_i32, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "hers_rerank_decrypt": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_i32, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "hers_load_secret_key": (c_i32, [c_vp, c_vp, c_vp]),
    "hers_encrypt_gallery": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_i32, c_i64, c_i64, c_u64, c_vp, c_vp, c_vp,
                                     ctypes.c_size_t, c_vp]),
    "hers_encrypt_probe": (c_i32, [c_vp, c_vp, c_i32, c_u64, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "hers_encrypt_probe_sk": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_u64, c_vp, c_u64, c_vp, c_vp, ctypes.c_size_t,
                                      c_vp]),
    "hers_import_gallery": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_i64, c_i64, c_vp, c_u64, c_vp]),
    "hers_import_probe": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_u64, c_vp]),
    "hers_export_gallery": (c_i32, [c_vp, c_vp, c_u64, c_i64, c_i32, c_i64, c_i64, c_vp, c_vp, ctypes.c_size_t,
                                    c_vp]),
    "hers_export_probe": (c_i32, [c_vp, c_vp, c_u64, c_i32, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "hers_search": (c_i32, [c_vp, c_vp, c_u64, c_i64, c_i32, c_vp, c_u64, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "hers_search_noalloc": (c_i32, [c_vp, c_vp, c_u64, c_i64, c_i32, c_vp, c_u64, c_vp, c_vp]),
    "hers_search_batch": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_vp), ctypes.POINTER(c_u64), ctypes.POINTER(c_i64),
                                  ctypes.POINTER(c_i32), ctypes.POINTER(c_vp), ctypes.POINTER(c_u64),
                                  ctypes.POINTER(c_vp), c_vp, ctypes.c_size_t, c_vp]),
    "hers_autotune_batch": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_vp), ctypes.POINTER(c_u64), ctypes.POINTER(c_i64),
                                    ctypes.POINTER(c_i32), ctypes.POINTER(c_vp), ctypes.POINTER(c_u64),
                                    ctypes.POINTER(c_vp), c_vp, ctypes.c_size_t, ctypes.c_int, c_vp,
                                    ctypes.POINTER(c_i64)]),
    "hers_plan_create": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_vp), ctypes.POINTER(c_u64), ctypes.POINTER(c_i64),
                                 ctypes.POINTER(c_i32), ctypes.POINTER(c_vp), ctypes.POINTER(c_u64),
                                 ctypes.POINTER(c_vp), c_vp, ctypes.c_size_t, ctypes.POINTER(c_vp)]),
    "hers_plan_launch": (c_i32, [c_vp, c_vp]),
    "hers_plan_destroy": (None, [c_vp]),
    "hers_decrypt_scores": (c_i32, [c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "hers_set_option": (c_i32, [c_vp, ctypes.c_char_p, c_i64]),
    "hers_autotune": (c_i32, [c_vp, c_vp, c_u64, c_i64, c_i32, c_vp, c_u64, c_vp, c_vp, ctypes.c_size_t,
                              ctypes.c_int, c_vp, ctypes.POINTER(c_i64)]),
    "hers_get_option": (c_i32, [c_vp, ctypes.c_char_p, ctypes.POINTER(c_i64)]),
    "hers_topk_workspace_bytes": (c_u64, [c_i64, c_i32]),
    "hers_topk": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "hers_profile_enable": (c_i32, [c_vp, c_i32]),
    "hers_profile_select": (c_i32, [c_vp, ctypes.c_char_p]),
    "hers_profile_read": (c_i32, [c_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_u64)]),
}

class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_i64), ("completed", c_i64), ("deferrals", c_i64), ("waves", c_i64),
                ("max_wave", c_i64), ("queued", c_i64), ("in_flight", c_i64), ("arena_peak", c_u64),
                ("gallery_bytes", c_u64)]


EXPORTS.update({
    "hers_server_create": (c_i32, [c_vp, c_vp, c_vp, ctypes.c_size_t, c_i32, ctypes.POINTER(c_vp)]),
    "hers_server_add_gallery": (c_i32, [c_vp, c_vp, c_u64, c_i64, c_i32, ctypes.POINTER(c_i32)]),
    "hers_server_submit": (c_i32, [c_vp, c_i32, c_vp, c_u64, ctypes.POINTER(c_i64)]),
    "hers_server_wait": (c_i32, [c_vp, c_i64, c_vp, c_vp, ctypes.POINTER(ctypes.c_double)]),
    "hers_server_stats_get": (c_i32, [c_vp, ctypes.POINTER(ServerStats)]),
    "hers_server_destroy": (None, [c_vp]),
})

OP_ENCRYPT_GALLERY, OP_ENCRYPT_PROBE, OP_SEARCH, OP_DECRYPT, OP_ENROLL, OP_SEARCH_LITERAL = 0, 1, 2, 3, 4, 5
OP_RERANK_ENCRYPT, OP_RERANK, OP_RERANK_DECRYPT, OP_EXPORT, OP_ENCRYPT_PROBE_SK = 6, 7, 8, 9, 10


class HersError(RuntimeError):
    pass


def declare(lib):
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def library(path=LIB_PATH):
    """Load libhers.so (built by paper_2003_12197_amd.build)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(path):
            raise HersError("libhers.so is not built (run paper_2003_12197_amd.build.build())")
        _LIB = declare(ctypes.CDLL(path))
    return _LIB


def make_params(n, qbits, t_bits, w_bits=0, d_max=128, feature_bound=63):
    p = HersParams()
    p.n, p.k, p.t_bits, p.w_bits, p.d_max, p.feature_bound = n, len(qbits), t_bits, w_bits, d_max, feature_bound
    for i, b in enumerate(qbits):
        p.qbits[i] = b
    return p


def _check(lib, rc, what):
    if rc != 0:
        raise HersError("%s failed (%d): %s" % (what, rc, lib.hers_last_error().decode()))


def resolve(n, qbits, t_bits, w_bits=0, d_max=128, feature_bound=63):
    """Host-only parameter resolution (no GPU)."""
    lib = library()
    info = HersInfo()
    _check(lib, lib.hers_params_resolve(ctypes.byref(make_params(n, qbits, t_bits, w_bits, d_max, feature_bound)),
                                        ctypes.byref(info)), "hers_params_resolve")
    return info


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _host_query(query):
    """A query as a contiguous host int32 array (the library reads it on the host)."""
    import numpy as np
    if isinstance(query, torch.Tensor):
        query = query.detach().cpu().numpy()
    return np.ascontiguousarray(query, dtype=np.int32).reshape(-1)


def _words(t):
    """Length of a search-form buffer in u32 words."""
    return t.numel() * t.element_size() // 4


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A libhers context on one GPU: parameters, tables and loaded keys."""

    def __init__(self, n, qbits, t_bits, w_bits=0, d_max=128, feature_bound=63, device=0):
        self.lib = library()
        self.device = torch.device("cuda", device)
        self.params = make_params(n, qbits, t_bits, w_bits, d_max, feature_bound)
        h = c_vp()
        _check(self.lib, self.lib.hers_ctx_create(ctypes.byref(self.params), device, ctypes.byref(h)),
               "hers_ctx_create")
        self.handle = h
        info = HersInfo()
        _check(self.lib, self.lib.hers_ctx_info(h, ctypes.byref(info)), "hers_ctx_info")
        self.info = info
        self.n, self.k, self.K, self.L = info.n, info.k, info.num_aux, info.num_digits
        self.q = [info.q[i] for i in range(info.k)]
        self.t = info.t

    def close(self):
        if self.handle:
            self.lib.hers_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- helpers
    def _empty(self, count, dtype):
        return torch.empty(int(count), dtype=dtype, device=self.device)

    def workspace(self, op, m, d):
        nbytes = int(self.lib.hers_workspace_bytes(self.handle, op, int(m), int(d)))
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)

    def blocks(self, m):
        return int(self.lib.hers_blocks(self.handle, int(m)))

    # ------------------------------------------------------------- calls
    def keygen(self, seed):
        """Returns (sk uint8 [n], pk int64 [2][k][n], rlk int64 [L][2][k][n]); keys are loaded."""
        n, k, L = self.n, self.k, self.L
        sk = self._empty(n, torch.uint8)
        pk = self._empty(2 * k * n, torch.int64).view(2, k, n)
        rlk = self._empty(L * 2 * k * n, torch.int64).view(L, 2, k, n)
        _check(self.lib, self.lib.hers_keygen(self.handle, seed, _ptr(sk), _ptr(pk), _ptr(rlk), _stream()),
               "hers_keygen")
        return sk, pk, rlk

    def load_keys(self, pk, rlk):
        _check(self.lib, self.lib.hers_load_keys(self.handle, _ptr(pk.contiguous()), _ptr(rlk.contiguous()),
                                                 _stream()), "hers_load_keys")

    def new_gallery(self, m, d):
        return self._empty(self.lib.hers_gallery_words(self.handle, int(m), int(d)), torch.int32)

    def encrypt_gallery(self, feats, m_total, seed, block0=0, nblocks=None, gallery=None, canon=None,
                        workspace=None):
        """feats: int32 [d][ld] on the device holding items block0*n ...; returns the search-form gallery."""
        d, ld = feats.shape
        M = self.blocks(m_total)
        if nblocks is None:
            nblocks = M - block0
        if gallery is None:
            gallery = self.new_gallery(m_total, d)
        if workspace is None:
            workspace = self.workspace(OP_ENCRYPT_GALLERY, nblocks * self.n, d)
        feats = feats.contiguous()
        _check(self.lib, self.lib.hers_encrypt_gallery(
            self.handle, _ptr(feats), ld, int(m_total), d, int(block0), int(nblocks), seed, _ptr(gallery),
            _ptr(canon), _ptr(workspace), workspace.numel(), _stream()), "hers_encrypt_gallery")
        return gallery

    def new_canonical(self, m, d):
        """Canonical gallery ciphertexts u64 [M][d][2][k][n] (uninitialised)."""
        return torch.empty((self.blocks(m), d, 2, self.k, self.n), dtype=torch.int64, device=self.device)

    def enroll_append(self, feats, k0, seed, gallery, canon, workspace=None):
        """Online enrollment of items k0 .. k0 + c - 1 (feats int32 [d][c] on the
        device) into a gallery of k0 items; updates canon and gallery in place."""
        d, c = feats.shape
        feats = feats.contiguous()
        need_g = int(self.lib.hers_gallery_words(self.handle, int(k0) + c, d))
        need_c = self.blocks(int(k0) + c) * d * 2 * self.k * self.n
        if gallery.numel() * gallery.element_size() < need_g * 4 or canon.numel() * canon.element_size() < need_c * 8:
            raise ValueError("gallery or canonical buffer does not cover item %d" % (int(k0) + c - 1))
        if workspace is None:
            workspace = self.workspace(OP_ENROLL, c, d)
        _check(self.lib, self.lib.hers_enroll_append(
            self.handle, _ptr(feats), c, int(k0), c, d, int(seed), _ptr(canon), _ptr(gallery),
            _ptr(workspace), workspace.numel(), _stream()), "hers_enroll_append")

    def encrypt_probe(self, query, seed, canon=None, probe=None, workspace=None):
        """query: int32 [d] (host array, or a tensor, copied to the host); returns the search-form probe."""
        q = _host_query(query)
        d = q.size
        if probe is None:
            probe = self._empty(self.lib.hers_probe_words(self.handle, d), torch.int32)
        if workspace is None and canon is None:
            workspace = self.workspace(OP_ENCRYPT_PROBE, 0, d)
        _check(self.lib, self.lib.hers_encrypt_probe(
            self.handle, q.ctypes.data_as(c_vp), d, seed, _ptr(probe), _ptr(canon), _ptr(workspace),
            0 if workspace is None else workspace.numel(), _stream()), "hers_encrypt_probe")
        return probe

    def encrypt_probe_sk(self, sk, query, seed, canon=None, probe=None, workspace=None):
        """query int32 [d] (host array or tensor) encrypted under the secret key (sk
        uint8 [n], or None for the loaded key); returns the search-form probe."""
        q = _host_query(query)
        d = q.size
        if probe is None:
            probe = self._empty(self.lib.hers_probe_words(self.handle, d), torch.int32)
        if workspace is None:
            workspace = self.workspace(OP_ENCRYPT_PROBE_SK, 0, d)
        _check(self.lib, self.lib.hers_encrypt_probe_sk(
            self.handle, _ptr(sk), q.ctypes.data_as(c_vp), d, int(seed), _ptr(probe), _words(probe), _ptr(canon),
            _ptr(workspace), workspace.numel(), _stream()), "hers_encrypt_probe_sk")
        return probe

    def new_scores(self, m):
        return self._empty(self.blocks(m) * 2 * self.k * self.n, torch.int64).view(-1, 2, self.k, self.n)

    def search(self, gallery, m, d, probe, scores=None, workspace=None):
        """Encrypted scores [M][2][k][n] (canonical)."""
        if scores is None:
            scores = self.new_scores(m)
        if workspace is None:
            workspace = self.workspace(OP_SEARCH, m, d)
        _check(self.lib, self.lib.hers_search(self.handle, _ptr(gallery), _words(gallery), int(m), int(d), _ptr(probe),
                                              _words(probe), _ptr(scores), _ptr(workspace), workspace.numel(),
                                              _stream()), "hers_search")
        return scores

    def search_noalloc(self, gallery, m, d, probe, scores):
        """hers_search with the library's static scratch array as workspace (no allocation)."""
        _check(self.lib, self.lib.hers_search_noalloc(self.handle, _ptr(gallery), _words(gallery), int(m), int(d),
                                                      _ptr(probe), _words(probe), _ptr(scores), _stream()),
               "hers_search_noalloc")
        return scores

    def search_literal(self, gallery, m, d, probe, scores=None, workspace=None):
        """The paper-literal per-dimension schedule (multiply, rescale, relinearize, add)."""
        if scores is None:
            scores = self.new_scores(m)
        if workspace is None:
            workspace = self.workspace(OP_SEARCH_LITERAL, m, d)
        _check(self.lib, self.lib.hers_search_literal(self.handle, _ptr(gallery), _words(gallery), int(m), int(d),
                                                      _ptr(probe), _words(probe), _ptr(scores), _ptr(workspace),
                                                      workspace.numel(), _stream()), "hers_search_literal")
        return scores

    # ---- canonical ciphertexts in and out of the search form
    def import_gallery(self, canon, m_total, d, block0=0, nblocks=None, gallery=None):
        """Canonical gallery ciphertexts of blocks block0 .. (int64 [nblocks][d][2][k][n] on
        the device) into the search form; returns the gallery."""
        if nblocks is None:
            nblocks = self.blocks(m_total) - block0
        if gallery is None:
            gallery = self.new_gallery(m_total, d)
        canon = canon.contiguous()
        _check(self.lib, self.lib.hers_import_gallery(self.handle, _ptr(canon), int(m_total), int(d), int(block0),
                                                      int(nblocks), _ptr(gallery), _words(gallery), _stream()),
               "hers_import_gallery")
        return gallery

    def import_probe(self, canon, d, probe=None):
        """Canonical probe ciphertexts (int64 [d][2][k][n]) into the search form."""
        if probe is None:
            probe = self._empty(self.lib.hers_probe_words(self.handle, int(d)), torch.int32)
        _check(self.lib, self.lib.hers_import_probe(self.handle, _ptr(canon.contiguous()), int(d), _ptr(probe),
                                                    _words(probe), _stream()), "hers_import_probe")
        return probe

    def export_gallery(self, gallery, m_total, d, block0=0, nblocks=None, out=None, workspace=None):
        """Search-form blocks block0 .. back to canonical ciphertexts [nblocks][d][2][k][n]."""
        if nblocks is None:
            nblocks = self.blocks(m_total) - block0
        if out is None:
            out = torch.empty((nblocks, d, 2, self.k, self.n), dtype=torch.int64, device=self.device)
        if workspace is None:
            workspace = self.workspace(OP_EXPORT, nblocks * self.n, d)
        _check(self.lib, self.lib.hers_export_gallery(self.handle, _ptr(gallery), _words(gallery), int(m_total),
                                                      int(d), int(block0), int(nblocks), _ptr(out), _ptr(workspace),
                                                      workspace.numel(), _stream()), "hers_export_gallery")
        return out

    def export_probe(self, probe, d, out=None, workspace=None):
        """Search-form probe back to canonical ciphertexts [d][2][k][n]."""
        if out is None:
            out = torch.empty((d, 2, self.k, self.n), dtype=torch.int64, device=self.device)
        if workspace is None:
            workspace = self.workspace(OP_EXPORT, 1, d)
        _check(self.lib, self.lib.hers_export_probe(self.handle, _ptr(probe), _words(probe), int(d), _ptr(out),
                                                    _ptr(workspace), workspace.numel(), _stream()),
               "hers_export_probe")
        return out

    # ---- two-stage search, second stage (packed 1:1 re-ranking)
    def rotation_keygen(self, seed, W):
        """Rotation keys for segments of W slots (canonical [log2 W][L][2][k][n]); loaded into the context."""
        rk = self._empty(self.lib.hers_rotation_key_words(self.handle, int(W)), torch.int64)
        _check(self.lib, self.lib.hers_rotation_keygen(self.handle, int(seed), int(W), _ptr(rk), _stream()),
               "hers_rotation_keygen")
        return rk

    def rerank_encrypt(self, feats, W, seed, replicate=False, canon=None):
        """Packed encryption of items (feats int32 [D][count]) or of a probe
        (feats [D][1], replicate=True); returns the search form [nct][K][2][n]."""
        D, count = feats.shape
        feats = feats.contiguous()
        nct = 1 if replicate else -(-count // (self.n // W))
        search = torch.empty((nct, self.K, 2, self.n), dtype=torch.int32, device=self.device)
        if canon is not None and canon.numel() * canon.element_size() < nct * 2 * self.k * self.n * 8:
            raise ValueError("canonical buffer too small")
        ws = self.workspace(OP_RERANK_ENCRYPT, nct, 0)
        _check(self.lib, self.lib.hers_rerank_encrypt(
            self.handle, _ptr(feats), count, count, D, int(W), int(bool(replicate)), int(seed), _ptr(search),
            _ptr(canon), _ptr(ws), ws.numel(), _stream()), "hers_rerank_encrypt")
        return search

    def rerank(self, items, ids, probe, W, out=None, workspace=None):
        """Encrypted scores of the probe against the ciphertexts `ids` (device int64) of `items`."""
        ids = ids.to(device=self.device, dtype=torch.int64).contiguous()
        nsel = ids.numel()
        if out is None:
            out = torch.empty((nsel, 2, self.k, self.n), dtype=torch.int64, device=self.device)
        if workspace is None:
            workspace = self.workspace(OP_RERANK, nsel, 0)
        _check(self.lib, self.lib.hers_rerank(self.handle, _ptr(items), items.shape[0], _ptr(ids), nsel, _ptr(probe),
                                              int(W), _ptr(out), _ptr(workspace), workspace.numel(), _stream()),
               "hers_rerank")
        return out

    def rerank_decrypt(self, sk, cts, W, out=None, workspace=None):
        """Client: int32 [nsel][n / W] scores of the segments of the re-rank ciphertexts."""
        nsel = cts.shape[0]
        if out is None:
            out = torch.empty((nsel, self.n // W), dtype=torch.int32, device=self.device)
        if workspace is None:
            workspace = self.workspace(OP_RERANK_DECRYPT, nsel, 0)
        _check(self.lib, self.lib.hers_rerank_decrypt(self.handle, _ptr(sk), _ptr(cts), nsel, int(W), _ptr(out),
                                                      _ptr(workspace), workspace.numel(), _stream()),
               "hers_rerank_decrypt")
        return out

    def batch_workspace(self, ms, blocks_per_round=None):
        """Workspace for search_batch: every request's accumulators for a round of blocks."""
        per = int(self.lib.hers_workspace_bytes(self.handle, OP_SEARCH, self.n, 1))
        rounds = blocks_per_round or max(self.blocks(m) for m in ms)
        return torch.empty(per * len(ms) * rounds, dtype=torch.uint8, device=self.device)

    def search_batch(self, galleries, ms, ds, probes, scores=None, workspace=None):
        nreq = len(galleries)
        if scores is None:
            scores = [self.new_scores(m) for m in ms]
        if workspace is None:
            workspace = self.batch_workspace(ms)
        arr = lambda ts: (c_vp * nreq)(*[t.data_ptr() for t in ts])
        words = lambda ts: (c_u64 * nreq)(*[_words(t) for t in ts])
        _check(self.lib, self.lib.hers_search_batch(
            self.handle, nreq, arr(galleries), words(galleries), (c_i64 * nreq)(*ms), (c_i32 * nreq)(*ds),
            arr(probes), words(probes), arr(scores), _ptr(workspace), workspace.numel(), _stream()),
            "hers_search_batch")
        return scores

    def autotune_batch(self, galleries, ms, ds, probes, scores, workspace, reps=2):
        """Pick the fastest multi-probe multiply-accumulate schedule for this batch; returns it."""
        nreq = len(galleries)
        arr = lambda ts: (c_vp * nreq)(*[t.data_ptr() for t in ts])
        words = lambda ts: (c_u64 * nreq)(*[_words(t) for t in ts])
        v = c_i64()
        _check(self.lib, self.lib.hers_autotune_batch(
            self.handle, nreq, arr(galleries), words(galleries), (c_i64 * nreq)(*ms), (c_i32 * nreq)(*ds),
            arr(probes), words(probes), arr(scores), _ptr(workspace), workspace.numel(), int(reps), _stream(),
            ctypes.byref(v)), "hers_autotune_batch")
        return v.value

    def plan(self, galleries, ms, ds, probes, scores, workspace):
        """Capture a batch as a HIP graph; returns a Plan whose launch() replays it."""
        nreq = len(galleries)
        arr = lambda ts: (c_vp * nreq)(*[t.data_ptr() for t in ts])
        words = lambda ts: (c_u64 * nreq)(*[_words(t) for t in ts])
        h = c_vp()
        _check(self.lib, self.lib.hers_plan_create(
            self.handle, nreq, arr(galleries), words(galleries), (c_i64 * nreq)(*ms), (c_i32 * nreq)(*ds),
            arr(probes), words(probes), arr(scores), _ptr(workspace), workspace.numel(), ctypes.byref(h)),
            "hers_plan_create")
        return Plan(self, h, (galleries, probes, scores, workspace))

    def set_option(self, key, value):
        _check(self.lib, self.lib.hers_set_option(self.handle, key.encode(), int(value)), "hers_set_option")

    def autotune(self, gallery, m, d, probe, reps=3, workspace=None, scores=None):
        """Pick the fastest multiply-accumulate schedule, NTT radix and (when a
        score buffer is given) overlap chunk count for this gallery; returns the schedule."""
        if workspace is None:
            workspace = self.workspace(OP_SEARCH, m, d)
        v = c_i64()
        _check(self.lib, self.lib.hers_autotune(self.handle, _ptr(gallery), _words(gallery), int(m), int(d),
                                                _ptr(probe), _words(probe),
                                                _ptr(scores) if scores is not None else None,
                                                _ptr(workspace), workspace.numel(), int(reps), _stream(),
                                                ctypes.byref(v)), "hers_autotune")
        return v.value

    def get_option(self, key):
        v = c_i64()
        _check(self.lib, self.lib.hers_get_option(self.handle, key.encode(), ctypes.byref(v)), "hers_get_option")
        return v.value

    def topk(self, scores, m, k):
        """(indices int64 [k], values int32 [k]) of the k highest decrypted scores."""
        idx = self._empty(k, torch.int64)
        val = self._empty(k, torch.int32)
        ws = torch.empty(max(256, int(self.lib.hers_topk_workspace_bytes(int(m), int(k)))), dtype=torch.uint8,
                         device=self.device)
        _check(self.lib, self.lib.hers_topk(self.handle, _ptr(scores), int(m), int(k), _ptr(idx), _ptr(val),
                                            _ptr(ws), ws.numel(), _stream()), "hers_topk")
        return idx, val

    def profile_enable(self, on=True):
        _check(self.lib, self.lib.hers_profile_enable(self.handle, 1 if on else 0), "hers_profile_enable")

    def profile_select(self, stages=None):
        """Time only the named stages (an iterable of names) while profiling; None: every stage."""
        arg = None if not stages else ",".join(stages).encode()
        _check(self.lib, self.lib.hers_profile_select(self.handle, arg), "hers_profile_select")

    def profile_read(self, stage):
        """(total ms, launches) of one stage since profile_enable."""
        ms, cnt = ctypes.c_double(), c_u64()
        _check(self.lib, self.lib.hers_profile_read(self.handle, stage.encode(), ctypes.byref(ms), ctypes.byref(cnt)),
               "hers_profile_read")
        return ms.value, cnt.value

    def load_secret_key(self, sk):
        """Keep sk's transform in the context; decrypt_scores(None, ...) then uses it."""
        _check(self.lib, self.lib.hers_load_secret_key(self.handle, _ptr(sk), _stream()), "hers_load_secret_key")

    def decrypt_scores(self, sk, scores, m, out=None, workspace=None):
        """int32 [m] decrypted scores (client side)."""
        if out is None:
            out = self._empty(m, torch.int32)
        if workspace is None:
            workspace = self.workspace(OP_DECRYPT, m, 1)
        _check(self.lib, self.lib.hers_decrypt_scores(self.handle, _ptr(sk), _ptr(scores), int(m), _ptr(out),
                                                      _ptr(workspace), workspace.numel(), _stream()),
               "hers_decrypt_scores")
        return out


class Plan:
    """A captured batch (hers_plan); keeps its buffers alive."""

    def __init__(self, ctx, handle, keep):
        self.ctx, self.handle, self._keep = ctx, handle, keep

    def launch(self):
        _check(self.ctx.lib, self.ctx.lib.hers_plan_launch(self.handle, _stream()), "hers_plan_launch")

    def close(self):
        if self.handle:
            self.ctx.lib.hers_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop (hers_server) on a context.

    The context belongs to the server's worker thread until close()."""

    def __init__(self, ctx, sk, arena_bytes, max_batch=16):
        import numpy as _np
        self._np = _np
        self.ctx, self.lib = ctx, ctx.lib
        self.sk = sk
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=ctx.device)
        torch.cuda.synchronize()
        h = c_vp()
        _check(self.lib, self.lib.hers_server_create(ctx.handle, _ptr(sk), _ptr(self.arena), self.arena.numel(),
                                                     max_batch, ctypes.byref(h)), "hers_server_create")
        self.handle = h
        self.galleries = {}
        self._tickets = {}

    def add_gallery(self, gallery, m, d):
        gid = c_i32()
        _check(self.lib, self.lib.hers_server_add_gallery(self.handle, _ptr(gallery), _words(gallery), int(m), int(d),
                                                          ctypes.byref(gid)), "hers_server_add_gallery")
        self.galleries[gid.value] = (gallery, int(m), int(d))
        return gid.value

    def submit(self, gid, query, seed):
        q = self._np.ascontiguousarray(query, dtype=self._np.int32)
        if q.ndim != 1 or q.size != self.galleries[gid][2]:
            raise ValueError("a query of %d values for a gallery of d = %d" % (q.size, self.galleries[gid][2]))
        t = c_i64()
        rc = self.lib.hers_server_submit(self.handle, gid, q.ctypes.data_as(c_vp), int(seed), ctypes.byref(t))
        _check(self.lib, rc, "hers_server_submit")
        self._tickets[t.value] = self.galleries[gid][1]
        return t.value

    def wait(self, ticket, scores=True, ciphertexts=False):
        """(latency ms, decrypted scores int32 [m] or None, score ciphertexts or None)."""
        gid_m = None
        lat = ctypes.c_double()
        out = ct = None
        # sizes come from the gallery of the ticket; the server checks the ticket
        if scores or ciphertexts:
            gid_m = self._ticket_sizes(ticket)
        if scores:
            out = self._np.empty(gid_m[0], dtype=self._np.int32)
        if ciphertexts:
            ct = self._np.empty(gid_m[1], dtype=self._np.uint64)
        rc = self.lib.hers_server_wait(self.handle, ticket, None if out is None else out.ctypes.data_as(c_vp),
                                       None if ct is None else ct.ctypes.data_as(c_vp), ctypes.byref(lat))
        self._tickets.pop(ticket, None)
        _check(self.lib, rc, "hers_server_wait")
        return lat.value, out, ct

    def _ticket_sizes(self, ticket):
        m = self._tickets[ticket]
        return m, self.ctx.blocks(m) * 2 * self.ctx.k * self.ctx.n

    def stats(self):
        s = ServerStats()
        _check(self.lib, self.lib.hers_server_stats_get(self.handle, ctypes.byref(s)), "hers_server_stats_get")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            self.lib.hers_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
