"""Log-structured block store oracle (O14) -- TEST INFRASTRUCTURE ONLY.

A plain model of the SSD tier of Sec. 3.4: the model is written once as an
immutable base segment; updated block versions are appended to patch
segments, never written in place; a per-block pointer

    Index[k] = (file_id, offset, size, version),   file_id 0 = the base,

names the newest version, and every read goes through it.  Compaction (off
the training path) rewrites the newest versions into a new base.

Two parts, sharing nothing with the library:

* ``LogStoreModel`` -- the store as in-memory byte segments.  Appends write
  the record and only then move Index[k] to it with version + 1 (so a record
  torn by a crash is never named); ``persist`` is the consistency barrier
  that makes the current Index the one a restart sees.
* ``read_persisted`` / ``read_block`` -- an independent reader of a store
  directory as the library lays it out: ``index.bin`` (three int64 K, record
  bytes, segment count, then K entries of int32 file_id, int32 pad, int64
  offset, size, version), ``base.seg`` and ``patch_NNNNNN.seg``.  The layout
  is the library's choice; the reader follows only the Index semantics above.
"""
from __future__ import annotations

import os
import struct

_ENTRY = struct.Struct("<iiqqq")   # file_id, pad, offset, size, version
_HEADER = struct.Struct("<qqq")    # K, record bytes, segment count


class LogStoreModel:
    """In-memory log-structured store over K blocks of ``rec`` bytes."""

    def __init__(self, base_records: list[bytes]):
        self.rec = len(base_records[0]) if base_records else 0
        assert all(len(r) == self.rec for r in base_records)
        self.K = len(base_records)
        self.segments: list[bytearray] = [bytearray(b"".join(base_records))]
        self.index = [(0, k * self.rec, self.rec, 0) for k in range(self.K)]
        self.persisted = list(self.index)
        self.new_patch()

    def new_patch(self) -> int:
        """Starts a patch segment; later appends go to it."""
        self.segments.append(bytearray())
        return len(self.segments) - 1

    def append(self, k: int, data: bytes) -> None:
        """Writes a new version of block k at the end of the current patch,
        then points Index[k] at it with the next version number."""
        assert len(data) == self.rec
        fid = len(self.segments) - 1
        off = len(self.segments[fid])
        self.segments[fid] += data
        self.index[k] = (fid, off, self.rec, self.index[k][3] + 1)

    def read(self, k: int, index=None) -> bytes:
        fid, off, size, _ = (index or self.index)[k]
        seg = self.segments[fid]
        assert off + size <= len(seg), "an index entry points past its segment"
        return bytes(seg[off:off + size])

    def persist(self) -> None:
        """Consistency barrier: the current Index becomes the one a restart
        reads."""
        self.persisted = list(self.index)

    def crash(self, torn_bytes: int = 0) -> None:
        """Loses the in-memory Index and cuts the last ``torn_bytes`` bytes of
        the current patch (an append in progress); the store reopens from
        the persisted Index with a fresh patch segment."""
        if torn_bytes:
            seg = self.segments[-1]
            del seg[max(0, len(seg) - torn_bytes):]
        self.index = list(self.persisted)
        self.new_patch()

    def compact(self) -> None:
        """Rewrites every block's newest version, in block order, as a new
        base segment; versions are kept and the patches are dropped."""
        base = bytearray(b"".join(self.read(k) for k in range(self.K)))
        self.index = [(0, k * self.rec, self.rec, self.index[k][3]) for k in range(self.K)]
        self.segments = [base]
        self.persist()
        self.new_patch()


def read_persisted(directory: str):
    """(K, record bytes, segment count, Index) of a store directory's
    persisted index file."""
    with open(os.path.join(directory, "index.bin"), "rb") as f:
        raw = f.read()
    K, rec, nseg = _HEADER.unpack_from(raw, 0)
    need = _HEADER.size + K * _ENTRY.size
    assert len(raw) >= need, "short index file"
    index = []
    for k in range(K):
        fid, _pad, off, size, ver = _ENTRY.unpack_from(raw, _HEADER.size + k * _ENTRY.size)
        index.append((fid, off, size, ver))
    return K, rec, nseg, index


def segment_path(directory: str, file_id: int) -> str:
    return os.path.join(directory, "base.seg" if file_id == 0 else f"patch_{file_id:06d}.seg")


def read_block(directory: str, index, k: int) -> bytes:
    """Block k's bytes as the Index names them, read straight from the
    segment file."""
    fid, off, size, _ = index[k]
    with open(segment_path(directory, fid), "rb") as f:
        f.seek(off)
        data = f.read(size)
    assert len(data) == size, f"block {k}: the index names bytes past the end of segment {fid}"
    return data
