// CPU check of the exception guard of the C ABI: each case runs a body that throws (or not)
// between FDX_ABI_TRY and FDX_ABI_CATCH and prints the status code and the message the guard
// left in the context's last-error buffer.
#include <cstdio>
#include <new>
#include <stdexcept>
#include <vector>

#include "abi_guard.h"

struct FakeCtx {
    char err[64] = {};
};

namespace fdx {
int abi_exception(FakeCtx *c) noexcept {
    return classify_exception(c ? c->err : nullptr, c ? sizeof c->err : 0);
}
}  // namespace fdx

static int bad_alloc_body(FakeCtx *c) {
    FDX_ABI_TRY
    throw std::bad_alloc();
    FDX_ABI_CATCH(c)
}

static int huge_vector_body(FakeCtx *c) {
    FDX_ABI_TRY
    std::vector<double> v;
    v.reserve(v.max_size());          // throws std::length_error or std::bad_alloc
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

static int runtime_error_body(FakeCtx *c) {
    FDX_ABI_TRY
    throw std::runtime_error("a long message that does not fit the sixty-four byte buffer of the fake context");
    FDX_ABI_CATCH(c)
}

static int int_body(FakeCtx *c) {
    FDX_ABI_TRY
    throw 7;
    FDX_ABI_CATCH(c)
}

static int ok_body(FakeCtx *c) {
    FDX_ABI_TRY
    return c ? FDX_OK : FDX_EINVAL;
    FDX_ABI_CATCH(c)
}

int main() {
    struct { const char *name; int (*f)(FakeCtx *); } cases[] = {
        {"bad_alloc", bad_alloc_body}, {"huge_vector", huge_vector_body},
        {"runtime_error", runtime_error_body}, {"int", int_body}, {"ok", ok_body}};
    for (auto &k : cases) {
        FakeCtx c;
        const int code = k.f(&c);
        std::printf("%s|%d|%s\n", k.name, code, c.err);
    }
    // no context: the guard still returns a code and writes nothing
    std::printf("null|%d|\n", bad_alloc_body(nullptr));
    return 0;
}
