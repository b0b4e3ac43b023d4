"""The guard that keeps stale counter figures out of the bench line: the
profile summaries record a hash of the sweep code with its comments removed,
so an edit to a comment keeps the figures and an edit to the code drops them
(`bench.py` then reports no traffic or VALU figure)."""

from paper_2001_05291_amd import profiling


def test_comments_and_layout_do_not_count():
    a = "int f(int x) {\n    // sum\n    return x + 1; /* one */\n}\n"
    b = "int f(int x)\n{\n    /* a longer\n       comment */\n    return x + 1;   // one more\n}\n"
    assert profiling.strip_comments(a) == profiling.strip_comments(b)


def test_code_and_literals_count():
    a = 'int f(int x) { return x + 1; }'
    assert profiling.strip_comments(a) != profiling.strip_comments(a.replace("+ 1", "+ 2"))
    s = 'const char *u = "a//b /* c */"; // tail'
    assert profiling.strip_comments(s) == 'const char *u = "a//b /* c */";'
    q = "char c = '\\''; char d = '/'; // x"
    assert profiling.strip_comments(q) == "char c = '\\''; char d = '/';"

