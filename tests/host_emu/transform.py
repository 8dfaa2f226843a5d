"""Source rewrite of the library's HIP sources for the CPU emulation build:
kernel launches `K<<<grid, block[, lds[, stream]]>>>(args)` become
`emu::launch(...)` calls (arguments evaluated at launch, as on the device),
dynamic LDS declarations read the emulator's buffer, and the workspace carver
leaves a poisoned 256-byte redzone after every buffer so that AddressSanitizer
reports an access that runs past one buffer into the next.
Usage: transform.py SRC_DIR OUT_DIR"""
import os
import re
import sys


def _match_back_angle(s, j):
    """s[j] == '>': index of the matching '<'."""
    depth = 0
    while j >= 0:
        if s[j] == '>':
            depth += 1
        elif s[j] == '<':
            depth -= 1
            if depth == 0:
                return j
        j -= 1
    raise ValueError("unbalanced template arguments")


def _match_paren(s, i):
    """s[i] == '(': index just past the matching ')'."""
    depth = 0
    while i < len(s):
        c = s[i]
        if c == '(':
            depth += 1
        elif c == ')':
            depth -= 1
            if depth == 0:
                return i + 1
        i += 1
    raise ValueError("unbalanced parentheses")


def _split_top(s):
    parts, depth, cur = [], 0, []
    for c in s:
        if c in '(<[{':
            depth += 1
        elif c in ')>]}':
            depth -= 1
        if c == ',' and depth == 0:
            parts.append(''.join(cur))
            cur = []
        else:
            cur.append(c)
    parts.append(''.join(cur))
    return [p.strip() for p in parts]


def rewrite_launches(s):
    out = []
    pos = 0
    while True:
        k = s.find('<<<', pos)
        if k < 0:
            out.append(s[pos:])
            return ''.join(out)
        # kernel expression before <<<
        j = k - 1
        while s[j].isspace():
            j -= 1
        end_name = j + 1
        if s[j] == '>':
            j = _match_back_angle(s, j) - 1
        while j >= 0 and (s[j].isalnum() or s[j] in '_:'):
            j -= 1
        start = j + 1
        kern = s[start:end_name]
        close = s.find('>>>', k)
        cfg = _split_top(s[k + 3:close])
        i = close + 3
        while s[i].isspace() or s[i] == '\\':
            i += 1
        assert s[i] == '(', kern
        args_end = _match_paren(s, i)
        args = s[i + 1:args_end - 1]
        while len(cfg) < 4:
            cfg.append('0' if len(cfg) == 2 else 'nullptr')
        call = (f"emu::launch(dim3({cfg[0]}), dim3({cfg[1]}), (size_t)({cfg[2]}), (hipStream_t)({cfg[3]}), "
                f"[](auto... a_) {{ {kern}(a_...); }}" + (f", {args})" if args.strip() else ")"))
        out.append(s[pos:start])
        out.append(call)
        pos = args_end


EXTERN_LDS = re.compile(r"extern\s+__shared__\s+(?:__align__\(\d+\)\s+)?([\w:]+(?:\s+[\w:]+)*?)\s+(\w+)\[\]\s*;")

CARVE_OLD = """        off = align_up(off + std::max<size_t>(bytes, 1));
        return base ? reinterpret_cast<P*>(base + o) : nullptr;"""
CARVE_NEW = """        off = align_up(off + std::max<size_t>(bytes, 1)) + 256;
        if (base) emu::poison(base + o + bytes, off - o - bytes);
        return base ? reinterpret_cast<P*>(base + o) : nullptr;"""


def rewrite(name, s, include_dir):
    s = EXTERN_LDS.sub(lambda m: f"{m.group(1)}* {m.group(2)} = ({m.group(1)}*)emu::dyn_lds();", s)
    s = rewrite_launches(s)
    if name == "api.hip":
        assert CARVE_OLD in s, "workspace carver changed: update the emulation rewrite"
        s = s.replace(CARVE_OLD, CARVE_NEW)
        s = s.replace('#include "../../include/modehr.h"', f'#include "{os.path.join(include_dir, "modehr.h")}"')
    return s


def main(src, dst, include_dir):
    os.makedirs(dst, exist_ok=True)
    for f in sorted(os.listdir(src)):
        if f.endswith((".hip", ".hpp")):
            t = rewrite(f, open(os.path.join(src, f)).read(), include_dir)
            name = f[:-4] + ".cpp" if f.endswith(".hip") else f
            open(os.path.join(dst, name), "w").write(t)


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2], sys.argv[3])
