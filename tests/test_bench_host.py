"""Host checks of bench.py that need no GPU."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_default_run_gives_the_training_leg_every_argument_it_reads():
    """The default run calls the 4M training leg with a Namespace of its own:
    it must carry every args.<name> that leg reads."""
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    fn = next(n for n in ast.walk(tree) if isinstance(n, ast.FunctionDef) and n.name == "bench_layered_training")
    used = {n.attr for n in ast.walk(fn) if isinstance(n, ast.Attribute) and isinstance(n.value, ast.Name)
            and n.value.id == "args"}
    calls = [n for n in ast.walk(tree) if isinstance(n, ast.Call) and isinstance(n.func, ast.Attribute)
             and n.func.attr == "Namespace"]
    assert calls, "no Namespace for the training leg"
    for c in calls:
        given = {k.arg for k in c.keywords}
        assert used <= given, f"missing {sorted(used - given)}"
