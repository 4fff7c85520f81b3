"""Loop-structure check on gfx950 assembly (hipcc -S output).

A persistent kernel hands rows out from a global counter: thread 0 takes the
next index with a returning 64-bit atomic add and stores it to an LDS slot
that the whole block then reads.  For the kernel to make progress, every
loop that contains a read of that slot must also contain the atomic;
otherwise the lanes in that loop re-read an index nobody advances.

The check reads the loop annotations LLVM writes beside each basic block
("This Loop Header", "in Loop: Header=", "Parent Loop"), finds the slot from
the first counter atomic and the LDS store of its result, and reports every
(kernel, block, loop) where a slot read sits in a loop without the atomic."""

import re

_ATOM = re.compile(r"global_atomic_add_x2 v\[\d+:\d+\], v\d+, v\[\d+:\d+\], s\[\d+:\d+\] sc0")
_DSW = re.compile(r"ds_write_b64 (v\d+), v\[\d+:\d+\](?: offset:(\d+))?")
_DSR = re.compile(r"ds_read_b64 v\[\d+:\d+\], (v\d+)(?: offset:(\d+))?")


def _functions(text):
    name, body = None, []
    for line in text.splitlines():
        m = re.match(r"^(_Z\w+):\s*;", line)
        if m:
            name, body = m.group(1), []
            continue
        if name is not None:
            body.append(line)
            if "s_endpgm" in line and not line.strip().startswith(";"):
                yield name, body
                name = None


def _blocks(lines):
    out, cur = [], None
    for ln in lines:
        m = re.match(r"^\.L(BB\d+_\d+):", ln) or re.match(r"^; %(bb\.\d+):", ln)
        if m or cur is None:
            cur = {"name": m.group(1) if m else "entry", "loop": None, "parents": [], "lines": []}
            out.append(cur)
        if re.search(r"=>\s*This (Inner )?Loop Header: Depth=\d+", ln):
            cur["loop"] = cur["name"]
        i = re.search(r"in Loop: Header=(BB\d+_\d+) Depth=\d+", ln)
        if i:
            cur["loop"] = i.group(1)
        p = re.search(r"Parent Loop (BB\d+_\d+) Depth=\d+", ln)
        if p:
            cur["parents"].append(p.group(1))
        cur["lines"].append(ln)
    return out


def _vgpr_const(flat, k, reg):
    """Value of VGPR `reg` before instruction k when, in layout order, it was
    last written by a move of an immediate; None otherwise."""
    num = int(reg[1:])
    for j in range(k - 1, -1, -1):
        parts = re.split(r"[\s,]+", flat[j][1].strip())
        if len(parts) < 2 or parts[0].startswith(("ds_write", "global_store", "global_atomic", "s_")):
            continue
        dst = parts[1]
        rng = re.match(r"v\[(\d+):(\d+)\]", dst)
        if dst == reg or (rng and int(rng.group(1)) <= num <= int(rng.group(2))):
            if parts[0] == "v_mov_b32_e32":
                try:
                    return int(parts[2], 0)
                except ValueError:
                    return None
            return None
    return None


def check(text):
    """Returns (number of persistent kernels found, list of violations)."""
    bad, kernels = [], 0
    for fname, lines in _functions(text):
        bl = _blocks(lines)
        parent = {b["name"]: b["parents"][-1] for b in bl if b["loop"] == b["name"] and b["parents"]}

        def chain(h):
            c = []
            while h:
                c.append(h)
                h = parent.get(h)
            return c

        flat = [(bi, ln) for bi, b in enumerate(bl) for ln in b["lines"] if not ln.strip().startswith(";")]
        slots = set()
        for k, (_, ln) in enumerate(flat):
            if not _ATOM.search(ln):
                continue
            for kk in range(k + 1, min(k + 14, len(flat))):
                m = _DSW.search(flat[kk][1])
                if m:
                    c = _vgpr_const(flat, kk, m.group(1))
                    if c is not None:
                        slots.add(c + int(m.group(2) or 0))
                    break
            break
        if not slots:
            continue
        kernels += 1
        # the counter may sit in different SGPRs at different fetches; these
        # kernels have no other returning 64-bit atomic add, so every one
        # counts as a fetch
        atom_loops = set()
        for bi, ln in flat:
            if _ATOM.search(ln):
                atom_loops.update(chain(bl[bi]["loop"]))
        for k, (bi, ln) in enumerate(flat):
            m = _DSR.search(ln)
            if not m:
                continue
            c = _vgpr_const(flat, k, m.group(1))
            if c is None or c + int(m.group(2) or 0) not in slots:
                continue
            for h in chain(bl[bi]["loop"]):
                if h not in atom_loops:
                    bad.append((fname, bl[bi]["name"], h))
    return kernels, bad
