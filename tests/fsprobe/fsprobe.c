/* File-open probe for the no-file-system test (LD_PRELOAD interposer).
 *
 * Interposes the libc entry points that open or create files and, while
 * recording is switched on (fsprobe_enable), writes one line per call to the
 * file named by FSPROBE_LOG: the path and the shared object that asked for it.
 * The asking object is the first frame of the call stack that lies outside
 * this probe and outside the C and C++ runtime libraries (libc, libstdc++,
 * libgcc_s, ld-linux), so that an open made by std::ifstream inside some
 * library is charged to that library rather than to libstdc++.
 *
 * Test infrastructure only: built from this source by the test that uses it.
 */
#define _GNU_SOURCE
#include <dlfcn.h>
#include <execinfo.h>
#include <fcntl.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

typedef int (*open_fn)(const char *, int, ...);
typedef int (*openat_fn)(int, const char *, int, ...);
typedef int (*creat_fn)(const char *, mode_t);
typedef FILE *(*fopen_fn)(const char *, const char *);
typedef int (*mkstemp_fn)(char *);
typedef char *(*mkdtemp_fn)(char *);

static int g_enabled;
static __thread int t_busy;

void fsprobe_enable(int on) { __atomic_store_n(&g_enabled, on, __ATOMIC_SEQ_CST); }

static int is_runtime_object(const char *name)
{
    static const char *skip[] = {"fsprobe", "libc.so", "libc-", "libstdc++", "libgcc_s", "ld-linux",
                                 "libpthread", "libm.so"};
    for (size_t i = 0; i < sizeof skip / sizeof skip[0]; ++i)
        if (strstr(name, skip[i])) return 1;
    return 0;
}

static void record(const char *fn, const char *path)
{
    if (!__atomic_load_n(&g_enabled, __ATOMIC_SEQ_CST) || t_busy) return;
    t_busy = 1;
    void *frames[64];
    int n = backtrace(frames, 64);
    const char *who = "?";
    for (int i = 0; i < n; ++i) {
        Dl_info info;
        if (dladdr(frames[i], &info) && info.dli_fname && !is_runtime_object(info.dli_fname)) {
            who = info.dli_fname;
            break;
        }
    }
    const char *log = getenv("FSPROBE_LOG");
    if (log) {
        /* written with the real open/write so that the probe does not record itself */
        static open_fn real_open;
        if (!real_open) real_open = (open_fn)dlsym(RTLD_NEXT, "open");
        int fd = real_open(log, O_WRONLY | O_CREAT | O_APPEND, 0644);
        if (fd >= 0) {
            char line[4096];
            int len = snprintf(line, sizeof line, "%s\t%s\t%s\n", fn, path ? path : "(null)", who);
            if (len > 0) {
                if (len > (int)sizeof line - 1) len = (int)sizeof line - 1;
                ssize_t w = write(fd, line, (size_t)len);
                (void)w;
            }
            close(fd);
        }
    }
    t_busy = 0;
}

#define REAL(name, type) \
    static type real_##name; \
    if (!real_##name) real_##name = (type)dlsym(RTLD_NEXT, #name)

static mode_t mode_arg(int flags, va_list ap)
{
    return (flags & (O_CREAT | O_TMPFILE)) ? (mode_t)va_arg(ap, int) : 0;
}

int open(const char *path, int flags, ...)
{
    va_list ap;
    va_start(ap, flags);
    mode_t m = mode_arg(flags, ap);
    va_end(ap);
    REAL(open, open_fn);
    record("open", path);
    return real_open(path, flags, m);
}

int open64(const char *path, int flags, ...)
{
    va_list ap;
    va_start(ap, flags);
    mode_t m = mode_arg(flags, ap);
    va_end(ap);
    REAL(open64, open_fn);
    record("open64", path);
    return real_open64(path, flags, m);
}

int openat(int dirfd, const char *path, int flags, ...)
{
    va_list ap;
    va_start(ap, flags);
    mode_t m = mode_arg(flags, ap);
    va_end(ap);
    REAL(openat, openat_fn);
    record("openat", path);
    return real_openat(dirfd, path, flags, m);
}

int openat64(int dirfd, const char *path, int flags, ...)
{
    va_list ap;
    va_start(ap, flags);
    mode_t m = mode_arg(flags, ap);
    va_end(ap);
    REAL(openat64, openat_fn);
    record("openat64", path);
    return real_openat64(dirfd, path, flags, m);
}

int creat(const char *path, mode_t mode)
{
    REAL(creat, creat_fn);
    record("creat", path);
    return real_creat(path, mode);
}

FILE *fopen(const char *path, const char *mode)
{
    REAL(fopen, fopen_fn);
    record("fopen", path);
    return real_fopen(path, mode);
}

FILE *fopen64(const char *path, const char *mode)
{
    REAL(fopen64, fopen_fn);
    record("fopen64", path);
    return real_fopen64(path, mode);
}

int mkstemp(char *tmpl)
{
    REAL(mkstemp, mkstemp_fn);
    record("mkstemp", tmpl);
    return real_mkstemp(tmpl);
}

char *mkdtemp(char *tmpl)
{
    REAL(mkdtemp, mkdtemp_fn);
    record("mkdtemp", tmpl);
    return real_mkdtemp(tmpl);
}
