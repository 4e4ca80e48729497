"""bench.py's modes run only on a GPU; this checks on the CPU that every
name a function of bench.py reads is bound somewhere it can see: its
parameters, its own or an enclosing function's assignments, loop and
comprehension targets, imports and nested definitions, the module's
globals, or the builtins."""
import ast
import builtins
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bound(node):
    """Names bound directly in a function body (not inside nested defs)."""
    out = set()
    a = node.args
    for arg in a.posonlyargs + a.args + a.kwonlyargs:
        out.add(arg.arg)
    if a.vararg:
        out.add(a.vararg.arg)
    if a.kwarg:
        out.add(a.kwarg.arg)
    stack = list(node.body)
    while stack:
        n = stack.pop()
        if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            out.add(n.name)
            continue
        if isinstance(n, ast.Lambda):
            continue
        if isinstance(n, ast.Name) and isinstance(n.ctx, (ast.Store, ast.Del)):
            out.add(n.id)
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            for al in n.names:
                out.add((al.asname or al.name).split(".")[0])
        elif isinstance(n, ast.ExceptHandler) and n.name:
            out.add(n.name)
        elif isinstance(n, (ast.Global, ast.Nonlocal)):
            out.update(n.names)
        stack.extend(ast.iter_child_nodes(n))
    return out


def _loads(node):
    """Names read directly in a function body (nested defs checked on their own)."""
    out = []
    stack = list(node.body) + list(node.args.defaults) + list(node.args.kw_defaults or [])
    while stack:
        n = stack.pop()
        if n is None:
            continue
        if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            stack.extend(n.decorator_list)
            stack.extend(n.args.defaults)
            continue
        if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load):
            out.append((n.id, n.lineno))
        stack.extend(ast.iter_child_nodes(n))
    return out


def _comprehension_targets(node):
    out = set()
    for n in ast.walk(node):
        if isinstance(n, ast.comprehension):
            for t in ast.walk(n.target):
                if isinstance(t, ast.Name):
                    out.add(t.id)
        if isinstance(n, ast.Lambda):
            for arg in n.args.args:
                out.add(arg.arg)
    return out


def test_bench_functions_read_only_bound_names():
    path = os.path.join(ROOT, "bench.py")
    tree = ast.parse(open(path).read(), path)
    module = set(dir(builtins))
    for n in tree.body:
        if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            module.add(n.name)
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            for al in n.names:
                module.add((al.asname or al.name).split(".")[0])
        else:
            for t in ast.walk(n):
                if isinstance(t, ast.Name) and isinstance(t.ctx, ast.Store):
                    module.add(t.id)
    missing = []

    def nested(fn):
        """Function definitions inside fn, not inside another nested one."""
        stack = list(fn.body)
        while stack:
            n = stack.pop()
            if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef)):
                yield n
                continue
            stack.extend(ast.iter_child_nodes(n))

    def visit(fn, enclosing):
        scope = enclosing | _bound(fn) | _comprehension_targets(fn)
        for name, line in _loads(fn):
            if name not in scope and name not in module:
                missing.append(f"{fn.name}:{line}: {name}")
        for inner in nested(fn):
            visit(inner, scope)

    for n in tree.body:
        if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef)):
            visit(n, set())
    assert not missing, missing
