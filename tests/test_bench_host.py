"""Host-side pieces of bench.py: the code hash that ties the recorded HBM
traffic figures to the kernels they were measured on."""
import bench


def test_code_text_ignores_comments_and_whitespace():
    a = "int f(int x) {  // doubles x\n  return 2 * x; /* the product */\n}\n"
    b = "// header comment\nint f(int x) {\n    return 2 * x;\n}"
    assert bench.code_text(a) == bench.code_text(b)


def test_code_text_sees_code_changes():
    a = "int f(int x) { return 2 * x; }"
    b = "int f(int x) { return 3 * x; }"
    assert bench.code_text(a) != bench.code_text(b)

