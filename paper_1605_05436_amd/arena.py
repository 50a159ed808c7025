"""Admission arena of the serving loop: a first-fit allocator over a byte
range of device memory (offsets only; the server owns the memory).

Pure host logic with no imports, so it can be loaded and tested without the
GPU library.
"""


class ArenaAllocator:
    """First-fit allocator over [0, size) with 256-byte granularity."""

    def __init__(self, size, align=256):
        self.align = align
        self.free = [(0, size)]          # sorted (offset, length)

    def alloc(self, nbytes):
        need = max(self.align, (nbytes + self.align - 1) // self.align * self.align)
        for i, (off, ln) in enumerate(self.free):
            if ln >= need:
                if ln == need:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + need, ln - need)
                return off, need
        return None, need

    def release(self, off, ln):
        free = self.free
        free.append((off, ln))
        free.sort()
        merged = [free[0]]
        for o, l in free[1:]:
            po, pl = merged[-1]
            if po + pl == o:
                merged[-1] = (po, pl + l)
            else:
                merged.append((o, l))
        self.free = merged
