"""Planting mistakes in the oracle (CPU only): a mutant of an oracle function is
its own source with one fragment replaced, compiled against the oracle module's
globals so that it sees (and, installed with monkeypatch, is seen by) the rest of
that module."""

import __future__
import inspect
import textwrap


def mutate(module, name: str, old: str, new: str):
    """Function `name` of `module` with the single occurrence of `old` replaced by `new`."""
    src = textwrap.dedent(inspect.getsource(getattr(module, name)))
    if src.count(old) != 1:
        raise AssertionError(f"{name}: fragment occurs {src.count(old)} times: {old!r}")
    code = compile(src.replace(old, new), f"<mutant of {module.__name__}.{name}>", "exec",
                   flags=__future__.annotations.compiler_flag, dont_inherit=True)
    local = {}
    exec(code, module.__dict__, local)
    return local[name]
