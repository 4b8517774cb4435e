"""Source-level guards on the hand-written HIP kernels (CPU only)."""
import glob
import os
import re

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2102_01734_amd", "csrc")


def _asm_strings():
    for path in sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.hpp"))):
        src = open(path).read()
        for m in re.finditer(r'\basm\s*(?:volatile\s*)?\(\s*((?:"(?:[^"\\]|\\.)*"\s*)+)', src):
            yield os.path.basename(path), "".join(re.findall(r'"((?:[^"\\]|\\.)*)"', m.group(1)))


def test_inline_readlanes_carry_their_wait_states():
    """A v_readlane / v_readfirstlane of a VGPR that the preceding vector instruction
    wrote needs wait states, which the compiler inserts only around instructions
    it generated itself: every such read written in inline asm starts with its own
    s_nop (a missing one read stale registers in the sweep kernel's visit weight)."""
    seen = 0
    for name, text in _asm_strings():
        lines = [l.strip() for l in text.replace("\\n", "\n").replace("\\t", " ").split("\n") if l.strip()]
        for i, line in enumerate(lines):
            if re.match(r"v_read(first)?lane", line):
                seen += 1
                assert i > 0 and re.match(r"s_nop\s+[1-9]", lines[i - 1]), (name, text)
    assert seen >= 1

